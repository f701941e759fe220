"""The C-ABI library loads and exports every entry point its header declares;
host-side argument checks reject bad configurations without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ktf.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ktf_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    import paper_1605_05508_amd as k
    if not os.path.exists(k.LIB_PATH):
        from paper_1605_05508_amd import build_lib
        build_lib.build()
    return k.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared()
    assert "ktf_fit" in names and "ktf_build" in names and "ktf_submit" in names
    for n in names:
        assert hasattr(lib, n), n
    import paper_1605_05508_amd as k
    assert sorted(k.EXPORTS) == names


def make_cfg(k, radii, **kw):
    arr = (C.c_double * len(radii))(*radii)
    base = dict(z_half=100.0, bz=3.8, sigma_r=0.01, sigma_rphi=0.01, sigma_z=0.1, n_zbins=64,
                n_phibins=512, max_cands=10, max_missed=1, n_seed_layers=3, chi2_cut=30.0,
                hbm_budget_bytes=1 << 30, max_inflight=8, x0=None, eloss=0.0, mass=0.13957)
    base.update(kw)
    x0 = None if base["x0"] is None else (C.c_double * len(radii))(*base["x0"])
    cfg = k._Config(len(radii), arr, base["z_half"], base["bz"], base["sigma_r"], base["sigma_rphi"],
                    base["sigma_z"], base["n_zbins"], base["n_phibins"], base["max_cands"],
                    base["max_missed"], base["n_seed_layers"], base["chi2_cut"],
                    base["hbm_budget_bytes"], base["max_inflight"], x0, base["eloss"], base["mass"])
    return cfg, (arr, x0)


@pytest.mark.parametrize("bad", [
    dict(radii=[4.0, 3.0, 8.0]),          # not increasing
    dict(radii=[]),                      # no layers
    dict(radii=[4.0] * 40),              # too many layers
    dict(sigma_r=0.0),                   # S would be singular
    dict(max_cands=0),
    dict(max_cands=99),
    dict(n_seed_layers=20),
    dict(n_zbins=0),
    dict(x0=[0.01] * 9 + [-0.01]),          # negative material
    dict(x0=[0.01] * 9 + [float("nan")]),   # not a number
    dict(x0=[0.01] * 10, mass=0.0),         # material needs a mass
    dict(x0=[0.01] * 10, eloss=-1.0),
])
def test_create_rejects_bad_config(lib, bad):
    import paper_1605_05508_amd as k
    radii = bad.pop("radii", [4.0 * (i + 1) for i in range(10)])
    cfg, arr = make_cfg(k, radii or [1.0], **bad)
    if not radii:
        cfg.n_layers = 0
    h = C.c_void_p()
    assert lib.ktf_create(C.byref(cfg), C.byref(h)) == k.EINVAL
    assert not h.value


def test_null_arguments(lib):
    import paper_1605_05508_amd as k
    assert lib.ktf_create(None, None) == k.EINVAL
    assert lib.ktf_destroy(None) == k.OK
    assert lib.ktf_last_error(None) == b""
    assert lib.ktf_fit(None, None, None, 0, None) == k.EINVAL
    assert lib.ktf_build(None, None, None, None) == k.EINVAL
    assert lib.ktf_submit(None, None, None) == k.EINVAL
    assert lib.ktf_poll(None, 0, None) == k.EINVAL
