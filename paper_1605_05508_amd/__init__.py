"""Python binding of libktf: batched Kalman-filter track fitting and building
on AMD MI355X (gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libktf.so`` behind the C-ABI declared in ``include/ktf.h``.
PyTorch provides device memory and streams.  There is no CPU fallback: if the
library is missing, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libktf.so")

OK, EINVAL, ENOMEM, EAGAIN, ENOTFOUND, EDEVICE = 0, -1, -2, -3, -4, -5
ST_NO_REACH, ST_S_NOT_PD, ST_NONFINITE = 1, 2, 4
FP64, FP32_BULK, FP32_PROP = 0, 1, 2
FIT_AUTO, FIT_FUSED, FIT_PERSISTENT, FIT_SWEEP, FIT_SWEEP_GRAPH = 0, 1, 2, 3, 4
MODES = {"auto": FIT_AUTO, "fused": FIT_FUSED, "persistent": FIT_PERSISTENT,
         "sweep": FIT_SWEEP, "sweep_graph": FIT_SWEEP_GRAPH}
PRECS = {"fp64": FP64, "fp32b": FP32_BULK, "fp32p": FP32_PROP}
MAX_LAYERS = 32

EXPORTS = ["ktf_create", "ktf_destroy", "ktf_last_error", "ktf_fit", "ktf_autotune_fit",
           "ktf_tuned_shape", "ktf_build", "ktf_bin_hits", "ktf_submit", "ktf_poll", "ktf_now",
           "ktf_serving_stats", "ktf_fit_noalloc", "ktf_debug_fail_next_event", "ktf_config_bytes"]
NOALLOC_SCRATCH_BYTES = 32 << 20


class KtfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libktf error {code}: {msg}")
        self.code = code


class _Config(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("layer_r", C.POINTER(C.c_double)), ("z_half", C.c_double),
                ("bz", C.c_double), ("sigma_r", C.c_double), ("sigma_rphi", C.c_double),
                ("sigma_z", C.c_double), ("n_zbins", C.c_int32), ("n_phibins", C.c_int32),
                ("max_cands", C.c_int32), ("max_missed", C.c_int32), ("n_seed_layers", C.c_int32),
                ("chi2_cut", C.c_double), ("hbm_budget_bytes", C.c_uint64),
                ("max_inflight", C.c_int32), ("layer_x0", C.POINTER(C.c_double)),
                ("eloss_per_x0", C.c_double), ("mass", C.c_double), ("seed_order", C.c_int32),
                ("n_etabins", C.c_int32), ("eta_max", C.c_double)]


class _FitIn(C.Structure):
    _fields_ = [("n", C.c_int64), ("pitch", C.c_int64), ("prec", C.c_int), ("seed_state", C.c_void_p),
                ("seed_cov", C.c_void_p), ("charge", C.c_void_p), ("hits", C.c_void_p),
                ("hit_valid", C.c_void_p), ("n_passes", C.c_int32)]


class _FitOut(C.Structure):
    _fields_ = [("state", C.c_void_p), ("cov", C.c_void_p), ("chi2", C.c_void_p),
                ("n_upd", C.c_void_p), ("status", C.c_void_p)]


class _EventBatch(C.Structure):
    _fields_ = [("n_events", C.c_int32), ("seed_off", C.POINTER(C.c_int64)),
                ("hit_off", C.POINTER(C.c_int64)), ("hit_pitch", C.c_int64), ("hits", C.c_void_p),
                ("seed_pitch", C.c_int64), ("seed_state", C.c_void_p), ("seed_cov", C.c_void_p),
                ("charge", C.c_void_p), ("seed_hit", C.c_void_p), ("prec", C.c_int)]


class _BuildOut(C.Structure):
    _fields_ = [("hit_idx", C.c_void_p), ("state", C.c_void_p), ("cov", C.c_void_p),
                ("chi2", C.c_void_p), ("n_hits", C.c_void_p), ("status", C.c_void_p),
                ("cand_hist", C.c_void_p), ("cand_count", C.c_void_p)]


class _EventHost(C.Structure):
    _fields_ = [("n_seeds", C.c_int64), ("hit_off", C.c_void_p), ("hits", C.c_void_p),
                ("seed_state", C.c_void_p), ("seed_cov", C.c_void_p), ("charge", C.c_void_p),
                ("seed_hit", C.c_void_p), ("prec", C.c_int)]


class _ResultHost(C.Structure):
    _fields_ = [("hit_idx", C.c_void_p), ("state", C.c_void_p), ("cov", C.c_void_p),
                ("chi2", C.c_void_p), ("n_hits", C.c_void_p), ("status", C.c_void_p),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libktf.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first (python -m paper_1605_05508_amd.build_lib)")
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.ktf_create.argtypes = [C.POINTER(_Config), C.POINTER(vp)]
    lib.ktf_destroy.argtypes = [vp]
    lib.ktf_last_error.argtypes = [vp]
    lib.ktf_last_error.restype = C.c_char_p
    lib.ktf_fit.argtypes = [vp, C.POINTER(_FitIn), C.POINTER(_FitOut), C.c_int, vp]
    lib.ktf_fit_noalloc.argtypes = [vp, C.POINTER(_FitIn), C.POINTER(_FitOut), C.c_int, vp]
    lib.ktf_autotune_fit.argtypes = [vp, C.POINTER(_FitIn), C.POINTER(_FitOut), vp]
    lib.ktf_tuned_shape.argtypes = [vp, C.c_int, C.c_int64, C.c_char_p, C.c_size_t]
    lib.ktf_build.argtypes = [vp, C.POINTER(_EventBatch), C.POINTER(_BuildOut), vp]
    lib.ktf_bin_hits.argtypes = [vp, C.POINTER(_EventBatch), vp, vp, vp]
    lib.ktf_submit.argtypes = [vp, C.POINTER(_EventHost), C.POINTER(C.c_uint64)]
    lib.ktf_poll.argtypes = [vp, C.c_uint64, C.POINTER(_ResultHost)]
    lib.ktf_now.argtypes = []
    lib.ktf_now.restype = C.c_double
    lib.ktf_serving_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]
    lib.ktf_debug_fail_next_event.argtypes = [vp]
    lib.ktf_config_bytes.argtypes = []
    lib.ktf_config_bytes.restype = C.c_size_t
    if lib.ktf_config_bytes() != C.sizeof(_Config):
        raise RuntimeError(f"{path} was built with a ktf_config of {lib.ktf_config_bytes()} bytes, "
                           f"this binding has {C.sizeof(_Config)}: rebuild the library")
    _lib = lib
    return lib


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libktf needs a ROCm GPU; none is visible")
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    """A libktf context on the current GPU for one detector and parameter set.

    radii: layer radii (cm); bz (T); sigma_r, sigma_rphi, sigma_z (cm);
    z_half (cm); n_zbins, n_phibins; max_cands, max_missed, n_seed_layers,
    chi2_cut; hbm_budget_bytes, max_inflight (serving).
    """

    def __init__(self, radii: Sequence[float], *, bz=3.8, sigma_r=0.01, sigma_rphi=0.01,
                 sigma_z=0.1, z_half=100.0, n_zbins=64, n_phibins=512, max_cands=10,
                 max_missed=1, n_seed_layers=3, chi2_cut=30.0, hbm_budget_bytes=8 << 30,
                 max_inflight=64, layer_x0=None, eloss_per_x0=0.0, mass=0.13957, seed_order=0,
                 n_etabins=0, eta_max=1.2):
        """layer_x0: per-layer material thickness in radiation lengths (a number
        for all layers, a sequence, or None for no material).  seed_order: 1
        to build on seeds sorted by their predicted cell with each wave's
        window box staged in LDS (results unchanged).  n_etabins > 0: bin hits
        in that many eta bins over |eta| < eta_max instead of n_zbins z bins
        (results unchanged)."""
        _torch()
        lib = load_library()
        self._lib = lib
        self.radii = [float(r) for r in radii]
        self.n_layers = len(self.radii)
        self._r = (C.c_double * max(1, self.n_layers))(*self.radii)
        self._x0 = None
        if layer_x0 is not None:
            x0 = [float(layer_x0)] * self.n_layers if isinstance(layer_x0, (int, float)) else \
                [float(v) for v in layer_x0]
            if len(x0) != self.n_layers:
                raise ValueError("layer_x0 needs one value per layer")
            self._x0 = (C.c_double * self.n_layers)(*x0)
        cfg = _Config(self.n_layers, self._r, z_half, bz, sigma_r, sigma_rphi, sigma_z, n_zbins,
                      n_phibins, max_cands, max_missed, n_seed_layers, chi2_cut,
                      int(hbm_budget_bytes), max_inflight, self._x0, eloss_per_x0, mass, int(seed_order),
                      int(n_etabins), float(eta_max))
        self.cfg = cfg
        self._ticket_dtype = {}
        h = C.c_void_p()
        rc = lib.ktf_create(C.byref(cfg), C.byref(h))
        if rc != OK:
            raise KtfError(rc, "ktf_create failed")
        self._h = h

    @classmethod
    def for_detector(cls, det, **kw):
        x0 = getattr(det, "x0", 0.0)
        if x0 > 0 and "layer_x0" not in kw:
            kw.update(layer_x0=x0, eloss_per_x0=det.eloss, mass=det.mass)
        return cls(det.radii, bz=det.bz, sigma_r=det.sigma_r, sigma_rphi=det.sigma_rphi,
                   sigma_z=det.sigma_z, z_half=det.z_half, **kw)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ktf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != OK:
            msg = self._lib.ktf_last_error(self._h)
            raise KtfError(rc, f"{what}: {msg.decode() if msg else ''}")

    # ---------------------------------------------------------------- fit
    def _fit_structs(self, state, cov, q, hits, valid, out, prec=None, passes=1):
        torch = _torch()
        if prec is None:
            prec = FP64 if state.dtype == torch.float64 else FP32_BULK
        else:
            prec = PRECS[prec]
            if (prec == FP64) != (state.dtype == torch.float64):
                raise ValueError("precision and storage dtype disagree")
        n = q.shape[0]
        pitch = state.shape[1]
        fin = _FitIn(n, pitch, prec, _ptr(state), _ptr(cov), _ptr(q), _ptr(hits), _ptr(valid), int(passes))
        fout = _FitOut(_ptr(out["state"]), _ptr(out["cov"]), _ptr(out["chi2"]), _ptr(out["nupd"]),
                       _ptr(out["status"]))
        return fin, fout

    def alloc_fit_out(self, n, pitch, dtype):
        torch = _torch()
        dev = torch.device("cuda")
        return dict(state=torch.empty((6, pitch), dtype=dtype, device=dev),
                    cov=torch.empty((21, pitch), dtype=dtype, device=dev),
                    chi2=torch.empty(pitch, dtype=torch.float64, device=dev),
                    nupd=torch.empty(pitch, dtype=torch.int32, device=dev),
                    status=torch.empty(pitch, dtype=torch.int32, device=dev))

    def fit(self, state, cov, q, hits, valid=None, *, mode="auto", out=None, stream=None, prec=None,
            passes=1):
        """Enqueue a fit.  state [6, pitch], cov [21, pitch] (float64 for the FP64
        path, float32 for the float-storage paths), q int8 [pitch] (first n =
        len(q) are tracks), hits [L, 3, pitch] same dtype, valid uint8 [L, pitch]
        or None.  prec: None (from the dtype: 'fp64' or 'fp32b') or 'fp32p'
        (float state propagation, double covariance; fused modes only).
        passes > 1: iterated refit (fused modes only)."""
        self._validate_fit(state, cov, q, hits, valid)
        if out is None:
            out = self.alloc_fit_out(q.shape[0], state.shape[1], state.dtype)
        fin, fout = self._fit_structs(state, cov, q, hits, valid, out, prec, passes)
        self._check(self._lib.ktf_fit(self._h, C.byref(fin), C.byref(fout), MODES[mode],
                                      _stream_handle(stream)), "ktf_fit")
        return out

    def fit_noalloc(self, state, cov, q, hits, valid=None, *, out, mode="fused", stream=None, prec=None,
                    passes=1):
        """ktf_fit_noalloc: the fit with the library allocating no device memory
        (scratch from its static per-GPU array).  The caller passes the outputs
        (see alloc_fit_out); modes 'auto', 'fused', 'persistent', 'sweep'."""
        self._validate_fit(state, cov, q, hits, valid)
        fin, fout = self._fit_structs(state, cov, q, hits, valid, out, prec, passes)
        self._check(self._lib.ktf_fit_noalloc(self._h, C.byref(fin), C.byref(fout), MODES[mode],
                                              _stream_handle(stream)), "ktf_fit_noalloc")
        return out

    def autotune_fit(self, state, cov, q, hits, valid=None, *, out=None, stream=None, prec=None):
        self._validate_fit(state, cov, q, hits, valid)
        if out is None:
            out = self.alloc_fit_out(q.shape[0], state.shape[1], state.dtype)
        fin, fout = self._fit_structs(state, cov, q, hits, valid, out, prec)
        self._check(self._lib.ktf_autotune_fit(self._h, C.byref(fin), C.byref(fout),
                                               _stream_handle(stream)), "ktf_autotune_fit")
        return out

    def tuned_shape(self, prec, n, trials=False):
        """The tuned launch shape for (prec, n) as a JSON string; with
        trials=True it keeps the time of every shape the tuner tried."""
        size = 8192
        buf = C.create_string_buffer(size)
        self._check(self._lib.ktf_tuned_shape(self._h, PRECS.get(prec, prec), n, buf, size),
                    "ktf_tuned_shape")
        d = json.loads(buf.value.decode())
        if not trials:
            d.pop("trials", None)
        return json.dumps(d)

    def _validate_fit(self, state, cov, q, hits, valid):
        torch = _torch()
        dt = state.dtype
        if dt not in (torch.float64, torch.float32):
            raise ValueError("state must be float64 (FP64) or float32 (FP32-bulk)")
        pitch = state.shape[1]
        L = self.n_layers
        if tuple(state.shape) != (6, pitch) or tuple(cov.shape) != (21, pitch):
            raise ValueError("state [6, pitch] and cov [21, pitch] expected")
        if tuple(hits.shape) != (L, 3, pitch) or hits.dtype != dt or cov.dtype != dt:
            raise ValueError(f"hits [{L}, 3, pitch] of the state's dtype expected")
        if q.dtype != torch.int8 or q.shape[0] > pitch:
            raise ValueError("q int8 [n <= pitch] expected")
        if valid is not None and (tuple(valid.shape) != (L, pitch) or valid.dtype != torch.uint8):
            raise ValueError(f"valid uint8 [{L}, pitch] expected")
        for t in (state, cov, q, hits) + ((valid,) if valid is not None else ()):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("inputs must be contiguous GPU tensors")

    # ------------------------------------------------------------ building
    def _batch(self, ev, prec):
        torch = _torch()
        seed_off = ev["seed_off"].astype("int64")
        hit_off = ev["hit_off"].astype("int64")
        self._keep = (seed_off, hit_off)
        b = _EventBatch(len(seed_off) - 1, seed_off.ctypes.data_as(C.POINTER(C.c_int64)),
                        hit_off.ctypes.data_as(C.POINTER(C.c_int64)), ev["hits"].shape[1],
                        _ptr(ev["hits"]), ev["state"].shape[1], _ptr(ev["state"]),
                        _ptr(ev["cov"]), _ptr(ev["q"]), _ptr(ev["seed_hit"]), prec)
        return b

    def build(self, ev, *, hist=False, stream=None, out=None):
        """Combinatorial building of a batch of events.

        ev: dict with host numpy seed_off [E+1], hit_off [E*L+1] and device
        tensors hits [3, hit_pitch], state [6, seed_pitch], cov [21,
        seed_pitch], q int8, seed_hit int32 [n_seed_layers, seed_pitch].
        """
        torch = _torch()
        dt = ev["state"].dtype
        prec = FP64 if dt == torch.float64 else FP32_BULK
        sp = ev["state"].shape[1]
        L = self.n_layers
        NC = self.cfg.max_cands
        dev = torch.device("cuda")
        if out is None:
            out = dict(hit_idx=torch.empty((L, sp), dtype=torch.int32, device=dev),
                       state=torch.empty((6, sp), dtype=dt, device=dev),
                       cov=torch.empty((21, sp), dtype=dt, device=dev),
                       chi2=torch.empty(sp, dtype=torch.float64, device=dev),
                       nhits=torch.empty(sp, dtype=torch.int32, device=dev),
                       status=torch.empty(sp, dtype=torch.int32, device=dev))
            if hist:
                out["hist"] = torch.empty((L, NC, 2, sp), dtype=torch.int32, device=dev)
                out["count"] = torch.empty((L, sp), dtype=torch.int32, device=dev)
        b = self._batch(ev, prec)
        bo = _BuildOut(_ptr(out["hit_idx"]), _ptr(out["state"]), _ptr(out["cov"]),
                       _ptr(out["chi2"]), _ptr(out["nhits"]), _ptr(out["status"]),
                       _ptr(out.get("hist")), _ptr(out.get("count")))
        self._check(self._lib.ktf_build(self._h, C.byref(b), C.byref(bo), _stream_handle(stream)),
                    "ktf_build")
        return out

    def bin_hits(self, ev, *, stream=None):
        torch = _torch()
        dt = ev["hits"].dtype
        prec = FP64 if dt == torch.float64 else FP32_BULK
        E = len(ev["seed_off"]) - 1
        nb = (self.cfg.n_etabins if self.cfg.n_etabins > 0 else self.cfg.n_zbins) * self.cfg.n_phibins
        dev = torch.device("cuda")
        offs = torch.empty((E * self.n_layers, nb + 1), dtype=torch.int32, device=dev)
        perm = torch.empty(ev["hits"].shape[1], dtype=torch.int32, device=dev)
        b = self._batch(ev, prec)
        self._check(self._lib.ktf_bin_hits(self._h, C.byref(b), _ptr(offs), _ptr(perm),
                                           _stream_handle(stream)), "ktf_bin_hits")
        return offs, perm

    # ------------------------------------------------------------- serving
    def submit(self, ev_host) -> int:
        """Queue one event from host numpy arrays: hit_off int64 [L+1], hits
        [3, nh], state [6, n], cov [21, n] (float64 for prec 'fp64', float32
        for 'fp32b'), q int8 [n], seed_hit int32 [nsl, n]."""
        import numpy as np
        prec = ev_host.get("prec", "fp32b")
        vt = np.float64 if prec == "fp64" else np.float32
        arrs = dict(hit_off=np.ascontiguousarray(ev_host["hit_off"], dtype=np.int64),
                    hits=np.ascontiguousarray(ev_host["hits"], dtype=vt),
                    state=np.ascontiguousarray(ev_host["state"], dtype=vt),
                    cov=np.ascontiguousarray(ev_host["cov"], dtype=vt),
                    q=np.ascontiguousarray(ev_host["q"], dtype=np.int8),
                    seed_hit=np.ascontiguousarray(ev_host["seed_hit"], dtype=np.int32))
        n = arrs["q"].shape[0]
        e = _EventHost(n, arrs["hit_off"].ctypes.data, arrs["hits"].ctypes.data,
                       arrs["state"].ctypes.data, arrs["cov"].ctypes.data, arrs["q"].ctypes.data,
                       arrs["seed_hit"].ctypes.data, PRECS[prec])
        t = C.c_uint64()
        self._check(self._lib.ktf_submit(self._h, C.byref(e), C.byref(t)), "ktf_submit")
        self._ticket_dtype[t.value] = vt
        return t.value

    def debug_fail_next_event(self):
        """Testing hook: the next submitted event fails at launch (host-forced)."""
        self._check(self._lib.ktf_debug_fail_next_event(self._h), "ktf_debug_fail_next_event")

    def poll(self, ticket, n_seeds):
        """Returns None while pending, else a dict of host numpy results
        (state and cov in the submitted event's precision)."""
        import numpy as np
        L = self.n_layers
        vt = self._ticket_dtype.get(ticket, np.float32)
        res = dict(hit_idx=np.empty((L, n_seeds), np.int32), state=np.empty((6, n_seeds), vt),
                   cov=np.empty((21, n_seeds), vt), chi2=np.empty(n_seeds, np.float64),
                   nhits=np.empty(n_seeds, np.int32), status=np.empty(n_seeds, np.uint32))
        r = _ResultHost(res["hit_idx"].ctypes.data, res["state"].ctypes.data, res["cov"].ctypes.data,
                        res["chi2"].ctypes.data, res["nhits"].ctypes.data, res["status"].ctypes.data,
                        0.0, 0.0, 0.0)
        rc = self._lib.ktf_poll(self._h, C.c_uint64(ticket), C.byref(r))
        if rc == EAGAIN:
            return None
        self._ticket_dtype.pop(ticket, None)
        self._check(rc, "ktf_poll")
        res.update(t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done)
        return res

    def serving_stats(self):
        q, f, d = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self._lib.ktf_serving_stats(self._h, C.byref(q), C.byref(f), C.byref(d)),
                    "ktf_serving_stats")
        return dict(queued=q.value, inflight=f.value, done=d.value)

    def now(self) -> float:
        return self._lib.ktf_now()
