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
    the diffuse-prior ndf 2 n - 5.  Their outputs amplify rounding without
    bound (chaotic), so parity for them is agreement of the divergence."""
    ndf = np.maximum(1, 2 * r["nupd"] - 5)
    return (r["status"] != 0) | (r["chi2"] / ndf >= 50)


def fp64_close(g, o, tol=1e-10, check_diverged=True, poor_tol=1e-6):
    """Per component |a-b| <= tol (|b| + sigma_i); cov |dP_ij| <= tol sqrt(P_ii P_jj)
    (+ a floor for entries that vanish); chi2 relative.  Diverged fits of the
    oracle must be diverged on the GPU too and are not compared value by value.
    Poorly fitted tracks (chi2/(2n-5) >= 5 on the oracle) stretch the
    linearisation and amplify rounding (measured up to ~5e-8 relative): they
    are held to poor_tol, with status and hit count exact."""
    bad = diverged(o)
    if check_diverged and bad.any():
        gd = (g["status"] != 0) | (g["chi2"] / np.maximum(1, 2 * g["nupd"] - 5) >= 10)
        assert np.all(gd[bad]), np.nonzero(bad & ~gd)
        keep = ~bad
        g = {k: v[..., keep] for k, v in g.items()}
        o = {k: v[..., keep] for k, v in o.items()}
    poor = o["chi2"] / np.maximum(1, 2 * o["nupd"] - 5) >= 5
    if poor.any() and poor_tol > tol:
        fp64_close({k: v[..., poor] for k, v in g.items()}, {k: v[..., poor] for k, v in o.items()},
                   poor_tol, False, poor_tol)
        g = {k: v[..., ~poor] for k, v in g.items()}
        o = {k: v[..., ~poor] for k, v in o.items()}
    sig = sigma_diag(o["cov"])
    ds = np.abs(g["state"] - o["state"])
    assert np.all(ds <= tol * (np.abs(o["state"]) + sig)), ds.max()
    diag = [0, 6, 11, 15, 18, 20]
    k = 0
    for i in range(6):
        for j in range(i, 6):
            scale = np.sqrt(np.abs(o["cov"][diag[i]] * o["cov"][diag[j]]))
            d = np.abs(g["cov"][k] - o["cov"][k])
            assert np.all(d <= tol * scale + 1e-300), (i, j, (d / scale).max())
            k += 1
    assert np.all(np.abs(g["chi2"] - o["chi2"]) <= tol * np.maximum(1.0, np.abs(o["chi2"])))
    assert np.array_equal(g["nupd"], o["nupd"])
    assert np.array_equal(g["status"].astype(np.uint32), o["status"])


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


def certified(o_dbg_n, o_dbg, o_margin, g_count, g_hist, tau):
    """Adjudication of a building mismatch of one seed: find the first layer
    whose kept (parent, hit) list differs; the mismatch is certified when
    the oracle's smallest decision gap at that layer is within tau."""
    L = o_dbg_n.shape[0]
    for l in range(L):
        n = o_dbg_n[l]
        if g_count[l] != n or not np.array_equal(g_hist[l, :n], o_dbg[l, :n]):
            return bool(o_margin[l] <= tau), l
    return True, -1
