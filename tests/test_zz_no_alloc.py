"""ktf_fit_noalloc, the fit for callers that cannot allocate, against ktf_fit.

Both entry points run the same kernels; the allocation-free one takes its
scratch (the persistent kernel's tile counter, the sweep's per-track end
layer and double positions) from a static per-GPU array instead of the
context's workspace.  So its outputs must equal ktf_fit's bit for bit, on
two calls in a row (the second smaller, over the scratch the first left
behind), and a sweep too large for the array must be refused."""
import numpy as np
import pytest

import trackgen as tg
from helpers import fit_inputs, pad_pitch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def k():
    import paper_1605_05508_amd as k
    return k


@pytest.fixture(scope="module")
def ctx(k):
    return k.Context(tg.barrel(10).radii)


def _bytes(out, n):
    return {key: v[..., :n].contiguous().cpu().numpy().view(np.uint8) for key, v in out.items()}


def _ragged_set(seed, n):
    rng = np.random.default_rng(seed)
    fs = tg.make_fit_set(rng, n, tg.barrel(10), pt_range=(0.5, 100.0), pt_log=True)
    v = fs.valid.copy()
    v[rng.random(v.shape) < 0.1] = 0
    v[0] = 1
    fs.valid = v
    return fs


CASES = [("fp64", "fused", 1), ("fp64", "persistent", 1), ("fp64", "sweep", 1), ("fp64", "auto", 1),
         ("fp32b", "fused", 1), ("fp32b", "persistent", 1), ("fp32b", "sweep", 1),
         ("fp32p", "persistent", 1), ("fp64", "persistent", 3)]


@pytest.mark.parametrize("prec,mode,passes", CASES)
def test_noalloc_equals_fit(ctx, k, prec, mode, passes):
    import torch
    sizes = [(61, 4000 + 17), (62, 1000 + 5)]  # the second call smaller than the first
    for seed, n in sizes:
        print(f"noalloc case prec={prec} mode={mode} passes={passes} seed={seed} n={n}", flush=True)
        fs = _ragged_set(seed, n)
        d = fit_inputs(fs, "fp64" if prec == "fp64" else "fp32b", pitch=pad_pitch(n) + 64)
        dt = d["state"].dtype
        ref = ctx.fit(d["state"], d["cov"], d["q"], d["hits"], d["valid"], mode=mode,
                      prec=prec, passes=passes)
        out = ctx.alloc_fit_out(n, d["state"].shape[1], dt)
        for v in out.values():
            v.fill_(0)  # a fill kernel; results must overwrite it
        ctx.fit_noalloc(d["state"], d["cov"], d["q"], d["hits"], d["valid"], out=out, mode=mode,
                        prec=prec, passes=passes)
        torch.cuda.synchronize()
        a, b = _bytes(ref, n), _bytes(out, n)
        for key in a:
            assert np.array_equal(a[key], b[key]), (prec, mode, n, key)


def test_noalloc_refuses_oversized_sweep(ctx, k):
    import torch
    n = 64
    pitch = k.NOALLOC_SCRATCH_BYTES // 25 + 4096  # float storage needs 25 bytes per track
    L = ctx.n_layers
    dev = torch.device("cuda")
    state = torch.zeros((6, pitch), dtype=torch.float32, device=dev)
    cov = torch.zeros((21, pitch), dtype=torch.float32, device=dev)
    q = torch.ones(n, dtype=torch.int8, device=dev)
    hits = torch.zeros((L, 3, pitch), dtype=torch.float32, device=dev)
    out = ctx.alloc_fit_out(n, pitch, torch.float32)
    with pytest.raises(k.KtfError) as ei:
        ctx.fit_noalloc(state, cov, q, hits, None, out=out, mode="sweep")
    assert ei.value.code == k.EINVAL and "scratch" in str(ei.value)
    with pytest.raises(k.KtfError) as ei:
        ctx.fit_noalloc(state, cov, q, hits, None, out=out, mode="sweep_graph")
    assert ei.value.code == k.EINVAL
