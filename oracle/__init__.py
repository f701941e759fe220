"""Plain FP64 CPU oracle for Kalman-filter track fitting and building.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the GPU library
and its Python binding never do.  It shares no code with the GPU path.

Thin ctypes wrapper around ``ktf_oracle.c`` (plain C, FP64, built with
``-O2 -fno-fast-math -ffp-contract=off``).  Inputs arrive in the boundary's
structure-of-arrays shapes (``state[6, n]``, ``cov[21, n]``,
``hits[L, 3, n]``) and are transposed here to the C code's per-track
layout.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ktf_oracle.c")
_LIB = os.path.join(_HERE, "libktf_oracle.so")
# The same source built with fused multiply-adds contracted wherever the
# compiler likes: it rounds differently at nearly every multiply-add, as a
# different compiler or device does.  Comparing the two builds measures the
# oracle's own rounding spread per track; GPU-parity tests hold a track to a
# small multiple of that spread where it exceeds the fixed FP64 tolerance.
_LIB_CONTRACT = os.path.join(_HERE, "libktf_oracle_contract.so")

NO_REACH = 1
S_NOT_PD = 2
NONFINITE = 4

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11"]


def _cpu_has_fma() -> bool:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("flags"):
                    return " fma " in line + " "
    except OSError:
        pass
    return False


def contract_cflags():
    """Flags of the contracted build: FMA contraction where the host has FMA
    (without it no contraction can happen and the two builds agree)."""
    return ["-O2", "-fno-fast-math", "-ffp-contract=fast", *(["-mfma"] if _cpu_has_fma() else []),
            "-fPIC", "-shared", "-std=c11"]


def build_lib(force: bool = True) -> str:
    """Compile the oracle shared library (and its contracted twin) with gcc."""
    for out, flags in ((_LIB, CFLAGS), (_LIB_CONTRACT, contract_cflags())):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            tmp = out + ".tmp"
            subprocess.check_call(["gcc", *flags, "-o", tmp, _SRC, "-lm", "-lpthread"])
            os.replace(tmp, out)
    return _LIB


class _Geom(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("radii", C.POINTER(C.c_double)), ("bz", C.c_double),
                ("sigma_r", C.c_double), ("sigma_rphi", C.c_double), ("sigma_z", C.c_double),
                ("x0", C.POINTER(C.c_double)), ("eloss", C.c_double), ("mass", C.c_double)]


class _BuildParams(C.Structure):
    _fields_ = [("max_cands", C.c_int32), ("max_missed", C.c_int32), ("chi2_cut", C.c_double),
                ("n_seed_layers", C.c_int32)]


_lib = None
_lib_contract = None


def lib(contract: bool = False):
    """The oracle library; contract=True: its contracted twin (see above)."""
    global _lib, _lib_contract
    if (_lib_contract if contract else _lib) is None:
        for path in (_LIB, _LIB_CONTRACT):
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
                build_lib(force=False)
        if contract:
            _lib_contract = C.CDLL(_LIB_CONTRACT)
        else:
            _lib = C.CDLL(_LIB)
    return _lib_contract if contract else _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _geom(det, material=True):
    """material=False fits as if the detector had no material (for tests
    that show what ignoring it costs)."""
    radii = _d(det.radii)
    x0 = getattr(det, "x0", 0.0)
    x0 = _d(np.broadcast_to(np.asarray(x0, dtype=np.float64), (len(det.radii),))) \
        if material and np.any(np.asarray(x0) > 0) else None
    g = _Geom(len(det.radii), _p(radii, C.c_double), det.bz, det.sigma_r, det.sigma_rphi,
              det.sigma_z, _p(x0, C.c_double), getattr(det, "eloss", 0.0), getattr(det, "mass", 0.13957))
    return g, (radii, x0)  # keep the arrays alive


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


# ------------------------------------------------------------- primitives

def transport(x, q, bz, s):
    out = np.zeros(6)
    lib().orc_transport(_p(_d(x), C.c_double), C.c_int(int(q)), C.c_double(bz), C.c_double(s),
                        _p(out, C.c_double))
    return out


def propagate(x, q, bz, r, nearest=False):
    """Returns (state at surface, 6x6 Jacobian, arc length, rc)."""
    xo = np.zeros(6)
    F = np.zeros(36)
    s = C.c_double(0.0)
    x = _d(x)
    rc = lib().orc_propagate(_p(x, C.c_double), C.c_int(int(q)), C.c_double(bz), C.c_double(r),
                             C.c_int(1 if nearest else 0), _p(xo, C.c_double),
                             _p(F, C.c_double), C.byref(s))
    return xo, F.reshape(6, 6), s.value, rc


def material(det, layer, x, P):
    """Material of one layer (see orc_material): returns (x', P' [6,6])."""
    g, keep = _geom(det)
    xo = np.zeros(6)
    Po = np.zeros(36)
    lib().orc_material(C.byref(g), C.c_int(int(layer)), _p(_d(x), C.c_double),
                       _p(_d(P).ravel(), C.c_double), _p(xo, C.c_double), _p(Po, C.c_double))
    return xo, Po.reshape(6, 6)


def cov_propagate(P, F):
    out = np.zeros(36)
    lib().orc_cov_propagate(_p(_d(P).ravel(), C.c_double), _p(_d(F).ravel(), C.c_double),
                            _p(out, C.c_double))
    return out.reshape(6, 6)


def hit_cov(m, sr, srphi, sz):
    V = np.zeros(9)
    lib().orc_hit_cov(_p(_d(m), C.c_double), C.c_double(sr), C.c_double(srphi), C.c_double(sz),
                      _p(V, C.c_double))
    return V.reshape(3, 3)


def update(xp, Pp, m, V):
    """Returns (x+, P+, chi2, rc)."""
    xo = np.zeros(6)
    Po = np.zeros(36)
    c2 = C.c_double(0.0)
    rc = lib().orc_update(_p(_d(xp), C.c_double), _p(_d(Pp).ravel(), C.c_double),
                          _p(_d(m), C.c_double), _p(_d(V).ravel(), C.c_double),
                          _p(xo, C.c_double), _p(Po, C.c_double), C.byref(c2))
    return xo, Po.reshape(6, 6), c2.value, rc


def chi2(xp, Pp, m, V):
    c2 = C.c_double(0.0)
    rc = lib().orc_chi2(_p(_d(xp), C.c_double), _p(_d(Pp).ravel(), C.c_double),
                        _p(_d(m), C.c_double), _p(_d(V).ravel(), C.c_double), C.byref(c2))
    return c2.value, rc


def unpack(p):
    """Packed 21 (first axis) -> [..., 6, 6]."""
    p = np.asarray(p)
    out = np.zeros(p.shape[1:] + (6, 6))
    k = 0
    for i in range(6):
        for j in range(i, 6):
            out[..., i, j] = p[k]
            out[..., j, i] = p[k]
            k += 1
    return out


def pack(P):
    P = np.asarray(P)
    return np.stack([P[..., i, j] for i in range(6) for j in range(i, 6)], axis=0)


# ------------------------------------------------------------------- fit

def fit_arrays(det, state, cov, q, hits, valid=None, nthreads=None, material=True, passes=1,
               contract=False):
    """Batched FP64 fit.  state[6,n], cov[21,n], q[n], hits[L,3,n], valid[L,n];
    passes > 1: iterated refit (orc_refit_track); contract=True: run the
    contracted build of the same oracle (to measure its rounding spread).

    Returns dict(state[6,n], cov[21,n], chi2[n], nupd[n], status[n]).
    """
    n = q.shape[0]
    L = len(det.radii)
    g, radii = _geom(det, material)
    st = _d(np.asarray(state).T)
    cv = _d(np.asarray(cov).T)
    qq = np.ascontiguousarray(q, dtype=np.int8)
    hh = _d(np.transpose(hits, (2, 0, 1)))
    vv = None if valid is None else np.ascontiguousarray(np.asarray(valid).T, dtype=np.uint8)
    so = np.zeros((n, 6))
    co = np.zeros((n, 21))
    c2 = np.zeros(n)
    nu = np.zeros(n, dtype=np.int32)
    stt = np.zeros(n, dtype=np.uint32)
    lib(contract).orc_fit_batch(C.byref(g), C.c_int64(n), _p(st, C.c_double), _p(cv, C.c_double),
                        _p(qq, C.c_int8), _p(hh, C.c_double), _p(vv, C.c_uint8),
                        _p(so, C.c_double), _p(co, C.c_double), _p(c2, C.c_double),
                        _p(nu, C.c_int32), _p(stt, C.c_uint32), C.c_int(int(passes)),
                        C.c_int(nthreads or default_threads()))
    return dict(state=so.T.copy(), cov=co.T.copy(), chi2=c2, nupd=nu, status=stt)


def fit(fs, nthreads=None, material=True, passes=1, contract=False):
    """Fit a trackgen.FitSet (passes > 1: iterated refit; contract: the
    contracted build)."""
    return fit_arrays(fs.det, fs.state, fs.cov, fs.q, fs.hits, fs.valid, nthreads, material, passes,
                      contract)


def carry_back(det, q, from_layer, x):
    """A state on layer from_layer carried back to layer 0 (orc_carry_back);
    returns (state, rc)."""
    g, keep = _geom(det)
    xo = np.zeros(6)
    rc = lib().orc_carry_back(C.byref(g), C.c_int(int(q)), C.c_int(int(from_layer)),
                              _p(_d(x), C.c_double), _p(xo, C.c_double))
    return xo, rc


# ---------------------------------------------------------------- binning

def bin_layer(hits, z_half, nz, nphi):
    """hits[3, n] -> (offsets[nz*nphi+1], perm[n])."""
    n = hits.shape[1]
    hh = _d(np.asarray(hits).T)
    offs = np.zeros(nz * nphi + 1, dtype=np.int32)
    perm = np.zeros(max(n, 1), dtype=np.int32)
    lib().orc_bin_layer(C.c_int64(n), _p(hh, C.c_double), C.c_double(z_half), C.c_int32(nz),
                        C.c_int32(nphi), _p(offs, C.c_int32), _p(perm, C.c_int32))
    return offs, perm[:n]


def eta(h):
    """Pseudorapidity of the point h = (x, y, z) seen from the origin."""
    f = lib().orc_eta
    f.restype = C.c_double
    return f(_p(_d(h), C.c_double))


def bin_layer_eta(hits, eta_max, neta, nphi):
    """hits[3, n] -> (offsets[neta*nphi+1], perm[n]) with rows of pseudorapidity."""
    n = hits.shape[1]
    hh = _d(np.asarray(hits).T)
    offs = np.zeros(neta * nphi + 1, dtype=np.int32)
    perm = np.zeros(max(n, 1), dtype=np.int32)
    lib().orc_bin_layer_eta(C.c_int64(n), _p(hh, C.c_double), C.c_double(eta_max), C.c_int32(neta),
                            C.c_int32(nphi), _p(offs, C.c_int32), _p(perm, C.c_int32))
    return offs, perm[:n]


# --------------------------------------------------------------- building

def build_event(bs, e, seeds=None, *, max_cands=10, max_missed=1, chi2_cut=30.0,
                n_seed_layers=3, nthreads=None, debug=False, contract=False):
    """Brute-force building of (a subset of) the seeds of event e of a BuildSet.

    seeds: indices local to the event (default all).  Returns dict of
    hit_idx[L, ns], state[6, ns], cov[21, ns], chi2, nhits, status and, with
    debug=True, dbg_n[L, ns], dbg[L, NC, 2, ns], margin[L + 1, ns] (per layer
    the smallest relative decision gap, then the final choice's).
    """
    det = bs.det
    L = det.n_layers
    g, radii = _geom(det)
    bp = _BuildParams(max_cands, max_missed, chi2_cut, n_seed_layers)
    ho = bs.hit_off[e * L:(e + 1) * L + 1]
    hits = _d(bs.hits[:, ho[0]:ho[-1]].T)
    loff = np.ascontiguousarray(ho - ho[0], dtype=np.int64)
    s0 = int(bs.seed_off[e])
    ns_ev = int(bs.seed_off[e + 1] - s0)
    idx = np.arange(ns_ev) if seeds is None else np.asarray(seeds)
    gi = s0 + idx
    n = idx.shape[0]
    st = _d(bs.state[:, gi].T)
    cv = _d(bs.cov[:, gi].T)
    qq = np.ascontiguousarray(bs.q[gi], dtype=np.int8)
    sh = np.ascontiguousarray(bs.seed_hit[:n_seed_layers, gi].T, dtype=np.int32)
    hit_idx = np.zeros((n, L), dtype=np.int32)
    so = np.zeros((n, 6))
    co = np.zeros((n, 21))
    c2 = np.zeros(n)
    nh = np.zeros(n, dtype=np.int32)
    stt = np.zeros(n, dtype=np.uint32)
    dn = np.zeros((n, L), dtype=np.int32) if debug else None
    dg = np.zeros((n, L, max_cands, 2), dtype=np.int32) if debug else None
    mg = np.zeros((n, L + 1)) if debug else None
    lib(contract).orc_build_event(C.byref(g), C.byref(bp), _p(hits, C.c_double), _p(loff, C.c_int64),
                          C.c_int64(n), _p(st, C.c_double), _p(cv, C.c_double),
                          _p(qq, C.c_int8), _p(sh, C.c_int32), _p(hit_idx, C.c_int32),
                          _p(so, C.c_double), _p(co, C.c_double), _p(c2, C.c_double),
                          _p(nh, C.c_int32), _p(stt, C.c_uint32), _p(dn, C.c_int32),
                          _p(dg, C.c_int32), _p(mg, C.c_double),
                          C.c_int(nthreads or default_threads()))
    out = dict(hit_idx=hit_idx.T.copy(), state=so.T.copy(), cov=co.T.copy(), chi2=c2,
               nhits=nh, status=stt)
    if debug:
        out.update(dbg_n=dn.T.copy(), dbg=np.transpose(dg, (1, 2, 3, 0)).copy(),
                   margin=mg.T.copy())
    return out
