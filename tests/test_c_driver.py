"""The C-ABI driven from a plain host program (tests/c/fit_from_c.cpp: HIP
runtime for device memory, no Python or torch): the FP64 fit it returns
equals the oracle's, in the fused and the graph-replayed sweep modes.
Without a device the program must fail cleanly at ktf_create."""
import os
import subprocess

import numpy as np
import pytest

import trackgen as tg
from helpers import fp64_close, oracle_with_spread

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "fit_from_c")


def write_input(path, fs):
    det, n, L = fs.det, fs.n, fs.det.n_layers
    with open(path, "wb") as f:
        np.array([n, L], np.int32).tofile(f)
        np.array([det.bz, det.sigma_r, det.sigma_rphi, det.sigma_z, det.z_half], np.float64).tofile(f)
        np.asarray(det.radii, np.float64).tofile(f)
        for a in (fs.state, fs.cov, fs.hits):
            np.ascontiguousarray(a, np.float64).tofile(f)
        np.ascontiguousarray(fs.q, np.int8).tofile(f)
        np.ascontiguousarray(fs.valid, np.uint8).tofile(f)


def read_output(path, n):
    raw = open(path, "rb").read()
    o = 0
    out = {}
    for key, shape, dt in (("state", (6, n), np.float64), ("cov", (21, n), np.float64),
                           ("chi2", (n,), np.float64), ("nupd", (n,), np.int32),
                           ("status", (n,), np.uint32)):
        cnt = int(np.prod(shape))
        out[key] = np.frombuffer(raw, dt, cnt, o).reshape(shape)
        o += cnt * np.dtype(dt).itemsize
    assert o == len(raw)
    return out


def test_built():
    assert os.access(EXE, os.X_OK), "build() compiles tests/c/fit_from_c"


def test_fails_cleanly_without_a_device(tmp_path):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    fs = tg.config1(n=10)
    write_input(tmp_path / "in.bin", fs)
    r = subprocess.run([EXE, str(tmp_path / "in.bin"), str(tmp_path / "out.bin"), "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 1 and "ktf_create" in r.stderr, (r.returncode, r.stderr)


@pytest.mark.gpu
@pytest.mark.parametrize("mode", [1, 4])  # KTF_FIT_FUSED, KTF_FIT_SWEEP_GRAPH
def test_fit_from_c_matches_oracle(tmp_path, orc, mode):
    rng = np.random.default_rng(61)
    fs = tg.make_fit_set(rng, 777, tg.barrel(10), pt_range=(0.5, 10.0))
    write_input(tmp_path / "in.bin", fs)
    r = subprocess.run([EXE, str(tmp_path / "in.bin"), str(tmp_path / "out.bin"), str(mode)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    g = read_output(tmp_path / "out.bin", fs.n)
    o = orc.fit(fs)
    assert np.array_equal(g["status"], o["status"])
    assert np.array_equal(g["nupd"], o["nupd"])
    fp64_close(g, o, oracle_with_spread(orc, fs)[1])
