"""Python binding of libpks.so (ctypes).  Argument marshalling only.

Every step of the filter and smoother runs in the HIP kernels of libpks.so;
this module turns torch tensors (device memory) and torch streams into the
plain pointers of the C ABI (``include/pks.h``) and raises on error codes.
Importing it loads the library and fails loudly if it is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpks.so")

PKS_OK, PKS_E_ARG, PKS_E_UNSUPPORTED, PKS_E_WORKSPACE, PKS_E_HIP, PKS_E_NUMERIC = range(6)
PKS_FP64, PKS_MIXED_FP32 = 0, 1
STATUS_NAMES = {0: "PKS_OK", 1: "PKS_E_ARG", 2: "PKS_E_UNSUPPORTED", 3: "PKS_E_WORKSPACE",
                4: "PKS_E_HIP", 5: "PKS_E_NUMERIC"}

EXPORTED = ["pks_workspace_bytes", "pks_filter", "pks_smooth", "pks_filter_smooth",
            "pks_filter_batched", "pks_smooth_batched", "pks_plan_create", "pks_plan_launch",
            "pks_plan_destroy", "pks_autotune", "pks_read_numeric_status", "pks_last_error",
            "pks_version", "pks_profile_start", "pks_profile_stop", "pks_loglik", "pks_loglik_batched",
            "pks_workspace_bytes_tv", "pks_filter_tv", "pks_smooth_tv", "pks_filter_smooth_tv", "pks_loglik_tv",
            "pks_filter_tv_batched", "pks_smooth_tv_batched", "pks_loglik_tv_batched",
            "pks_hmm_workspace_bytes", "pks_hmm_filter", "pks_hmm_smooth", "pks_hmm_filter_smooth",
            "pks_filter_smooth_noalloc", "pks_noalloc_scratch_bytes", "pks_set_debug_poison",
            "pks_debug_poison", "pks_plan_create_tv", "pks_check_offsets"]


class PksError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


class pks_model(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("F", ctypes.c_void_p), ("u", ctypes.c_void_p), ("Q", ctypes.c_void_p),
                ("H", ctypes.c_void_p), ("d", ctypes.c_void_p), ("R", ctypes.c_void_p),
                ("m0", ctypes.c_void_p), ("P0", ctypes.c_void_p),
                ("per_sequence", ctypes.c_int32)]


class pks_hmm(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("Pi", ctypes.c_void_p), ("p0", ctypes.c_void_p)]


class pks_model_tv(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("F", ctypes.c_void_p), ("u", ctypes.c_void_p), ("Q", ctypes.c_void_p),
                ("H", ctypes.c_void_p), ("d", ctypes.c_void_p), ("R", ctypes.c_void_p),
                ("m0", ctypes.c_void_p), ("P0", ctypes.c_void_p), ("per_sequence", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libpks.so not found at %s: build it with "
                          "`python -m paper_1905_13002_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    mp = ctypes.POINTER(pks_model)
    mt = ctypes.POINTER(pks_model_tv)
    hp = ctypes.POINTER(pks_hmm)
    sig = {
        "pks_hmm_workspace_bytes": (sz, [i32, i64]),
        "pks_filter_smooth_noalloc": (ctypes.c_int, [mp, i64, vp, vp, vp, vp, vp, ctypes.c_int, vp]),
        "pks_noalloc_scratch_bytes": (sz, []),
        "pks_set_debug_poison": (ctypes.c_int, [i32]),
        "pks_check_offsets": (ctypes.c_int, [i32, vp, i64, vp, ctypes.POINTER(i32), vp]),
        "pks_debug_poison": (i32, []),
        "pks_hmm_filter": (ctypes.c_int, [hp, i64, vp, vp, vp, vp, sz, vp]),
        "pks_hmm_smooth": (ctypes.c_int, [hp, i64, vp, vp, vp, sz, vp]),
        "pks_hmm_filter_smooth": (ctypes.c_int, [hp, i64, vp, vp, vp, vp, vp, sz, vp]),
        "pks_workspace_bytes_tv": (sz, [i32, i32, i64, ctypes.c_int]),
        "pks_filter_tv": (ctypes.c_int, [mt, i64, vp, vp, vp, ctypes.c_int, vp, sz, vp]),
        "pks_smooth_tv": (ctypes.c_int, [mt, i64, vp, vp, vp, vp, ctypes.c_int, vp, sz, vp]),
        "pks_filter_smooth_tv": (ctypes.c_int, [mt, i64, vp, vp, vp, vp, vp, ctypes.c_int, vp, sz, vp]),
        "pks_loglik_tv": (ctypes.c_int, [mt, i64, vp, vp, vp, vp, vp, i32, ctypes.c_int, vp, sz, vp]),
        "pks_filter_tv_batched": (ctypes.c_int, [mt, i32, vp, i64, vp, vp, vp, ctypes.c_int, vp, sz, vp]),
        "pks_smooth_tv_batched": (ctypes.c_int, [mt, i32, vp, i64, vp, vp, vp, vp, ctypes.c_int, vp, sz, vp]),
        "pks_loglik_tv_batched": (ctypes.c_int, [mt, i32, vp, i64, vp, vp, vp, vp, vp, i32, ctypes.c_int, vp, sz,
                                                 vp]),
        "pks_workspace_bytes": (sz, [i32, i32, i64, i32, ctypes.c_int]),
        "pks_filter": (ctypes.c_int, [mp, i64, vp, vp, vp, ctypes.c_int, vp, sz, vp]),
        "pks_smooth": (ctypes.c_int, [mp, i64, vp, vp, vp, vp, ctypes.c_int, vp, sz, vp]),
        "pks_filter_smooth": (ctypes.c_int, [mp, i64, vp, vp, vp, vp, vp, ctypes.c_int, vp, sz, vp]),
        "pks_filter_batched": (ctypes.c_int, [mp, i32, vp, i64, vp, vp, vp, ctypes.c_int, vp, sz, vp]),
        "pks_smooth_batched": (ctypes.c_int, [mp, i32, vp, i64, vp, vp, vp, vp, ctypes.c_int, vp, sz, vp]),
        "pks_plan_create": (ctypes.c_int, [mp, i32, vp, i64, vp, vp, vp, vp, vp, ctypes.c_int, vp, sz,
                                           ctypes.c_char_p, vp, ctypes.POINTER(vp)]),
        "pks_plan_create_tv": (ctypes.c_int, [mt, i32, vp, i64, vp, vp, vp, vp, vp, ctypes.c_int, vp, sz,
                                              ctypes.c_char_p, vp, ctypes.POINTER(vp)]),
        "pks_loglik": (ctypes.c_int, [mp, i64, vp, vp, vp, vp, vp, i32, ctypes.c_int, vp, sz, vp]),
        "pks_loglik_batched": (ctypes.c_int, [mp, i32, vp, i64, vp, vp, vp, vp, vp, i32, ctypes.c_int, vp, sz,
                                              vp]),
        "pks_plan_launch": (ctypes.c_int, [vp, vp]),
        "pks_plan_destroy": (ctypes.c_int, [vp]),
        "pks_autotune": (ctypes.c_int, [i32, i32, i32, i64, ctypes.c_int, ctypes.c_char_p, vp]),
        "pks_read_numeric_status": (ctypes.c_int, [vp, ctypes.POINTER(i32), vp]),
        "pks_last_error": (ctypes.c_char_p, []),
        "pks_profile_start": (ctypes.c_int, []),
        "pks_profile_stop": (ctypes.c_int, [i32, ctypes.c_char_p, ctypes.POINTER(ctypes.c_float),
                                             ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "pks_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(status: int):
    if status != PKS_OK:
        raise PksError(status, lib.pks_last_error().decode())


def _prec(precision) -> int:
    if precision in (PKS_FP64, "fp64", "f64", torch.float64):
        return PKS_FP64
    if precision in (PKS_MIXED_FP32, "mixed", "fp32", "f32", torch.float32):
        return PKS_MIXED_FP32
    raise ValueError("precision must be 'fp64' or 'mixed'")


def _rdtype(prec: int):
    return torch.float64 if prec == PKS_FP64 else torch.float32


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class DeviceModel:
    """A model's matrices as float64 device tensors (kept alive with the struct)."""
    F: torch.Tensor
    Q: torch.Tensor
    H: torch.Tensor
    R: torch.Tensor
    m0: torch.Tensor
    P0: torch.Tensor
    u: Optional[torch.Tensor] = None
    d: Optional[torch.Tensor] = None
    per_sequence: bool = False
    time_varying: bool = False      # F, Q, H, R, u, d hold one row per step

    @property
    def nx(self):
        return self.F.shape[-1]

    @property
    def ny(self):
        return self.H.shape[-2]

    def struct(self):
        s = pks_model_tv() if self.time_varying else pks_model()
        s.nx, s.ny = self.nx, self.ny
        for f in ("F", "Q", "H", "R", "m0", "P0", "u", "d"):
            t = getattr(self, f)
            setattr(s, f, None if t is None else t.data_ptr())
        s.per_sequence = 1 if self.per_sequence else 0
        return s


def to_device(model, device="cuda", per_sequence: bool = False, time_varying: bool = False) -> DeviceModel:
    """Copy a workloads.Model (numpy) to the device as float64 tensors."""
    cv = lambda a: None if a is None else torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(device)
    return DeviceModel(cv(model.F), cv(model.Q), cv(model.H), cv(model.R), cv(model.m0), cv(model.P0),
                       cv(model.u), cv(model.d), per_sequence, time_varying)


def workspace_bytes(nx: int, ny: int, total: int, B: int = 1, precision="fp64", time_varying=False) -> int:
    if time_varying:
        n = lib.pks_workspace_bytes_tv(nx, ny, int(total), _prec(precision))
    else:
        n = lib.pks_workspace_bytes(nx, ny, int(total), int(B), _prec(precision))
    if n == 0:
        raise PksError(PKS_E_ARG, "invalid problem shape")
    return int(n)


def workspace(nx, ny, total, B=1, precision="fp64", device="cuda", time_varying=False) -> torch.Tensor:
    return torch.empty(workspace_bytes(nx, ny, total, B, precision, time_varying), dtype=torch.uint8,
                       device=device)


def _ws_for(model: "DeviceModel", total, B, prec, device):
    return workspace(model.nx, model.ny, total, B, prec, device, model.time_varying)


def _out(shape, prec, device):
    return torch.empty(shape, dtype=_rdtype(prec), device=device)


def filter(model: DeviceModel, y: torch.Tensor, precision="fp64", ws=None, out=None, stream=None):
    """Parallel Kalman filter: returns (m [T,nx], P [T,nx,nx])."""
    prec = _prec(precision)
    T = y.shape[0]
    m, P = out if out is not None else (_out((T, model.nx), prec, y.device),
                                         _out((T, model.nx, model.nx), prec, y.device))
    ws = ws if ws is not None else _ws_for(model, T, 1, prec, y.device)
    ms = model.struct()
    fn = lib.pks_filter_tv if model.time_varying else lib.pks_filter
    _check(fn(ctypes.byref(ms), T, _ptr(y), _ptr(m), _ptr(P), prec, _ptr(ws), ws.numel(), _stream(stream)))
    return m, P


def smooth(model: DeviceModel, m: torch.Tensor, P: torch.Tensor, precision="fp64", ws=None, out=None,
           stream=None):
    """Parallel RTS smoother from filtered moments: returns (ms, Ps)."""
    prec = _prec(precision)
    T = m.shape[0]
    ms_, Ps_ = out if out is not None else (torch.empty_like(m), torch.empty_like(P))
    ws = ws if ws is not None else _ws_for(model, T, 1, prec, m.device)
    st = model.struct()
    fn = lib.pks_smooth_tv if model.time_varying else lib.pks_smooth
    _check(fn(ctypes.byref(st), T, _ptr(m), _ptr(P), _ptr(ms_), _ptr(Ps_), prec, _ptr(ws), ws.numel(),
              _stream(stream)))
    return ms_, Ps_


def filter_smooth(model: DeviceModel, y: torch.Tensor, precision="fp64", ws=None, out=None, stream=None):
    """Filter then smoother in one call: returns (m, P, ms, Ps)."""
    prec = _prec(precision)
    T = y.shape[0]
    nx = model.nx
    if out is None:
        out = (_out((T, nx), prec, y.device), _out((T, nx, nx), prec, y.device),
               _out((T, nx), prec, y.device), _out((T, nx, nx), prec, y.device))
    m, P, ms_, Ps_ = out
    ws = ws if ws is not None else _ws_for(model, T, 1, prec, y.device)
    st = model.struct()
    fn = lib.pks_filter_smooth_tv if model.time_varying else lib.pks_filter_smooth
    _check(fn(ctypes.byref(st), T, _ptr(y), _ptr(m), _ptr(P), _ptr(ms_), _ptr(Ps_), prec, _ptr(ws), ws.numel(),
              _stream(stream)))
    return m, P, ms_, Ps_


def filter_batched(model: DeviceModel, offsets: torch.Tensor, y: torch.Tensor, precision="fp64", ws=None,
                   out=None, stream=None):
    prec = _prec(precision)
    B = offsets.shape[0] - 1
    total = y.shape[0]
    nx = model.nx
    m, P = out if out is not None else (_out((total, nx), prec, y.device), _out((total, nx, nx), prec, y.device))
    ws = ws if ws is not None else _ws_for(model, total, B, prec, y.device)
    st = model.struct()
    fn = lib.pks_filter_tv_batched if model.time_varying else lib.pks_filter_batched
    _check(fn(ctypes.byref(st), B, _ptr(offsets), total, _ptr(y), _ptr(m), _ptr(P), prec, _ptr(ws), ws.numel(),
              _stream(stream)))
    return m, P


def smooth_batched(model: DeviceModel, offsets: torch.Tensor, m: torch.Tensor, P: torch.Tensor,
                   precision="fp64", ws=None, out=None, stream=None):
    prec = _prec(precision)
    B = offsets.shape[0] - 1
    total = m.shape[0]
    ms_, Ps_ = out if out is not None else (torch.empty_like(m), torch.empty_like(P))
    ws = ws if ws is not None else _ws_for(model, total, B, prec, m.device)
    st = model.struct()
    fn = lib.pks_smooth_tv_batched if model.time_varying else lib.pks_smooth_batched
    _check(fn(ctypes.byref(st), B, _ptr(offsets), total, _ptr(m), _ptr(P), _ptr(ms_), _ptr(Ps_), prec, _ptr(ws),
              ws.numel(), _stream(stream)))
    return ms_, Ps_


def loglik(model: DeviceModel, y: torch.Tensor, m: torch.Tensor, P: torch.Tensor, precision="fp64",
           cumulative=False, steps=True, ws=None, stream=None):
    """Marginal likelihood from filter outputs: returns (ll [T] or None, total [1]).

    ll holds log p(y_k | y_1:k-1), or log p(y_1:k) when ``cumulative``;
    total is log p(y_1:T).  ``steps=False`` skips ll (total only)."""
    prec = _prec(precision)
    T = y.shape[0]
    ll = torch.empty(T, dtype=torch.float64, device=y.device) if (steps or cumulative) else None
    tot = torch.empty(1, dtype=torch.float64, device=y.device)
    ws = ws if ws is not None else _ws_for(model, T, 1, prec, y.device)
    st = model.struct()
    fn = lib.pks_loglik_tv if model.time_varying else lib.pks_loglik
    _check(fn(ctypes.byref(st), T, _ptr(y), _ptr(m), _ptr(P), _ptr(ll), _ptr(tot), 1 if cumulative else 0, prec,
              _ptr(ws), ws.numel(), _stream(stream)))
    return ll, tot


def loglik_batched(model: DeviceModel, offsets: torch.Tensor, y: torch.Tensor, m: torch.Tensor,
                   P: torch.Tensor, precision="fp64", cumulative=False, steps=True, ws=None, stream=None):
    """Batched marginal likelihood: returns (ll [total] or None, totals [B])."""
    prec = _prec(precision)
    B = offsets.shape[0] - 1
    total = y.shape[0]
    ll = torch.empty(total, dtype=torch.float64, device=y.device) if (steps or cumulative) else None
    tot = torch.empty(B, dtype=torch.float64, device=y.device)
    ws = ws if ws is not None else _ws_for(model, total, B, prec, y.device)
    st = model.struct()
    fn = lib.pks_loglik_tv_batched if model.time_varying else lib.pks_loglik_batched
    _check(fn(ctypes.byref(st), B, _ptr(offsets), total, _ptr(y), _ptr(m), _ptr(P), _ptr(ll), _ptr(tot),
              1 if cumulative else 0, prec, _ptr(ws), ws.numel(), _stream(stream)))
    return ll, tot


class Plan:
    """A captured filter + smoother (HIP graph) bound to fixed buffers; time-varying
    models (to_device(..., time_varying=True)) capture their per-step precompute too."""

    def __init__(self, model: DeviceModel, y: torch.Tensor, offsets: Optional[torch.Tensor] = None,
                 precision="fp64", tune_cache: Optional[str] = None, stream=None):
        prec = _prec(precision)
        self.prec = prec
        self.model = model
        self.y = y
        self.offsets = offsets
        total = y.shape[0]
        B = 1 if offsets is None else offsets.shape[0] - 1
        nx = model.nx
        dev = y.device
        self.m = _out((total, nx), prec, dev)
        self.P = _out((total, nx, nx), prec, dev)
        self.ms = _out((total, nx), prec, dev)
        self.Ps = _out((total, nx, nx), prec, dev)
        self.ws = workspace(nx, model.ny, total, B, prec, dev, model.time_varying)
        self._struct = model.struct()
        h = ctypes.c_void_p()
        create = lib.pks_plan_create_tv if model.time_varying else lib.pks_plan_create
        _check(create(ctypes.byref(self._struct), B, _ptr(offsets), total, _ptr(y), _ptr(self.m),
                                   _ptr(self.P), _ptr(self.ms), _ptr(self.Ps), prec, _ptr(self.ws),
                                   self.ws.numel(), tune_cache.encode() if tune_cache else None, _stream(stream),
                                   ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(lib.pks_plan_launch(self.handle, _stream(stream)))
        return self.m, self.P, self.ms, self.Ps

    def close(self):
        if self.handle:
            lib.pks_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(nx, ny, B, total, precision="fp64", cache_path: Optional[str] = None, stream=None):
    _check(lib.pks_autotune(nx, ny, B, int(total), _prec(precision),
                            cache_path.encode() if cache_path else None, _stream(stream)))


def check_offsets(offsets: torch.Tensor, total: int, ws: Optional[torch.Tensor] = None, stream=None):
    """Checks device offsets [B+1] against the packing rules (synchronises):
    returns (True, -1), or (False, the smallest offending index)."""
    B = offsets.shape[0] - 1
    ws = ws if ws is not None else torch.empty(256, dtype=torch.uint8, device=offsets.device)
    bad = ctypes.c_int32(-1)
    st = lib.pks_check_offsets(B, _ptr(offsets), int(total), _ptr(ws), ctypes.byref(bad), _stream(stream))
    if st == PKS_E_ARG and bad.value >= 0:
        return False, int(bad.value)
    _check(st)
    return True, -1


def set_debug_poison(on: bool):
    """Debug mode: every call first fills its workspace's floating-point
    regions with NaN (see pks_set_debug_poison)."""
    _check(lib.pks_set_debug_poison(1 if on else 0))


def debug_poison() -> bool:
    return bool(lib.pks_debug_poison())


def read_numeric_status(ws: torch.Tensor, stream=None):
    """Returns (ok, first_bad_sequence or -1); clears the flag."""
    bad = ctypes.c_int32(-1)
    st = lib.pks_read_numeric_status(_ptr(ws), ctypes.byref(bad), _stream(stream))
    if st == PKS_E_NUMERIC:
        return False, int(bad.value)
    _check(st)
    return True, -1


def profile_start():
    _check(lib.pks_profile_start())


def profile_stop(max_kernels: int = 64):
    """Returns {kernel name: (total ms, launches)} recorded since profile_start()."""
    names = ctypes.create_string_buffer(64 * max_kernels)
    tot = (ctypes.c_float * max_kernels)()
    cnt = (ctypes.c_int32 * max_kernels)()
    n = ctypes.c_int32(0)
    _check(lib.pks_profile_stop(max_kernels, names, tot, cnt, ctypes.byref(n)))
    out = {}
    for i in range(n.value):
        nm = names.raw[64 * i:64 * (i + 1)].split(b"\0", 1)[0].decode()
        out[nm] = (float(tot[i]), int(cnt[i]))
    return out


# ---------------------------------------------------------------------------
# discrete-state hidden Markov model
# ---------------------------------------------------------------------------
@dataclass
class DeviceHmm:
    """Transition matrix Pi [K,K] and prior p0 [K] as float64 device tensors."""
    Pi: torch.Tensor
    p0: torch.Tensor

    @property
    def K(self):
        return self.Pi.shape[-1]

    def struct(self):
        s = pks_hmm()
        s.K = self.K
        s.Pi = self.Pi.data_ptr()
        s.p0 = self.p0.data_ptr()
        return s


def hmm_to_device(Pi, p0, device="cuda") -> DeviceHmm:
    cv = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(device)
    return DeviceHmm(cv(Pi), cv(p0))


def hmm_workspace(K: int, T: int, device="cuda") -> torch.Tensor:
    n = lib.pks_hmm_workspace_bytes(K, int(T))
    if n == 0:
        raise PksError(PKS_E_ARG, "invalid HMM workspace request (K=%d, T=%d)" % (K, T))
    return torch.empty(n, dtype=torch.uint8, device=device)


def hmm_filter_smooth(model: DeviceHmm, L: torch.Tensor, ws=None, out=None, smooth=True, stream=None):
    """Filtered marginals alpha [T,K], log p(y_1:k) [T] and (``smooth``) the
    smoothed marginals gamma [T,K] from the emission log-likelihoods L [T,K]."""
    T, K = L.shape[0], model.K
    if L.dtype != torch.float64 or L.ndim != 2 or L.shape[1] != K:
        raise ValueError("L must be float64 [T, K]")
    ws = ws if ws is not None else hmm_workspace(K, T, L.device)
    if out is None:
        alpha = torch.empty((T, K), dtype=torch.float64, device=L.device)
        logp = torch.empty(T, dtype=torch.float64, device=L.device)
        gamma = torch.empty((T, K), dtype=torch.float64, device=L.device) if smooth else None
    else:
        alpha, logp, gamma = out
    st = model.struct()
    if smooth:
        _check(lib.pks_hmm_filter_smooth(ctypes.byref(st), T, _ptr(L), _ptr(alpha), _ptr(logp), _ptr(gamma),
                                         _ptr(ws), ws.numel(), _stream(stream)))
    else:
        _check(lib.pks_hmm_filter(ctypes.byref(st), T, _ptr(L), _ptr(alpha), _ptr(logp), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return alpha, logp, gamma


def hmm_smooth(model: DeviceHmm, alpha: torch.Tensor, ws=None, out=None, stream=None):
    """Smoothed marginals gamma [T,K] from filtered marginals alpha [T,K]."""
    T, K = alpha.shape[0], model.K
    ws = ws if ws is not None else hmm_workspace(K, T, alpha.device)
    gamma = out if out is not None else torch.empty((T, K), dtype=torch.float64, device=alpha.device)
    st = model.struct()
    _check(lib.pks_hmm_smooth(ctypes.byref(st), T, _ptr(alpha), _ptr(gamma), _ptr(ws), ws.numel(),
                              _stream(stream)))
    return gamma


def version() -> str:
    return lib.pks_version().decode()
