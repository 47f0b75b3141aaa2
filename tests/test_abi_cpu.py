"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, sizes workspaces, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pks.h")

pks = pytest.importorskip("paper_1905_13002_amd.pks", reason="libpks.so not built")
lib = pks.lib


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pks_[a-z_]+)\s*\(", txt)))


def test_header_symbols_exported():
    names = declared_functions()
    assert "pks_filter" in names and "pks_smooth" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(pks.EXPORTED) == set(names)


def test_version():
    assert "pks" in pks.version()


def test_workspace_bytes():
    n1 = lib.pks_workspace_bytes(4, 2, 1024, 1, 0)
    n2 = lib.pks_workspace_bytes(4, 2, 1 << 20, 1, 0)
    n3 = lib.pks_workspace_bytes(4, 2, 1 << 20, 1, 1)
    assert 0 < n1 < n2 and 0 < n3 < n2
    assert lib.pks_workspace_bytes(4, 2, 0, 1, 0) > 0
    for bad in ((0, 2, 10, 1, 0), (65, 2, 10, 1, 0), (4, 0, 10, 1, 0), (4, 65, 10, 1, 0),
                (4, 2, -1, 1, 0), (4, 2, 10, 0, 0), (4, 2, 10, 1, 7)):
        assert lib.pks_workspace_bytes(*bad) == 0
    # batched workspaces hold one constant block per model
    assert lib.pks_workspace_bytes(4, 2, 10000, 4096, 0) > lib.pks_workspace_bytes(4, 2, 10000, 1, 0)


FAKE = 0x10000000   # never dereferenced: every case below fails validation first


def fake_model(nx=4, ny=2, per_sequence=0, **null):
    m = pks.pks_model()
    m.nx, m.ny = nx, ny
    for i, f in enumerate(("F", "Q", "H", "R", "m0", "P0")):
        setattr(m, f, None if null.get(f) else FAKE + 0x100000 * (i + 1))
    m.u = m.d = None
    m.per_sequence = per_sequence
    return m


def call_filter(model, T=16, y=FAKE + 0x1000000, m=FAKE + 0x2000000, P=FAKE + 0x3000000, prec=0,
                ws=FAKE + 0x8000000, ws_bytes=None):
    if ws_bytes is None:
        ok = model is not None and 1 <= model.nx <= 64 and 1 <= model.ny <= 64 and prec in (0, 1)
        ws_bytes = lib.pks_workspace_bytes(model.nx, model.ny, max(T, 0), 1, prec) if ok else 1 << 30
    mp = ctypes.byref(model) if model is not None else None
    return lib.pks_filter(mp, T, y, m, P, prec, ws, ws_bytes, None)


def test_filter_argument_errors():
    assert call_filter(None) == pks.PKS_E_ARG
    assert call_filter(fake_model(nx=0)) == pks.PKS_E_ARG
    assert call_filter(fake_model(nx=65)) == pks.PKS_E_ARG
    assert call_filter(fake_model(ny=0)) == pks.PKS_E_ARG
    assert call_filter(fake_model(F=True)) == pks.PKS_E_ARG
    assert call_filter(fake_model(R=True)) == pks.PKS_E_ARG
    assert call_filter(fake_model(), T=-1) == pks.PKS_E_ARG
    assert call_filter(fake_model(), y=None) == pks.PKS_E_ARG
    assert call_filter(fake_model(), P=None) == pks.PKS_E_ARG
    assert call_filter(fake_model(), prec=3) == pks.PKS_E_ARG
    assert call_filter(fake_model(), ws=None) == pks.PKS_E_ARG
    assert call_filter(fake_model(per_sequence=1)) == pks.PKS_E_ARG
    assert "per_sequence" in lib.pks_last_error().decode()


def test_filter_aliasing_rejected():
    # m overlapping y, P overlapping m
    assert call_filter(fake_model(), y=FAKE + 0x1000000, m=FAKE + 0x1000000 + 8) == pks.PKS_E_ARG
    assert call_filter(fake_model(), m=FAKE + 0x2000000, P=FAKE + 0x2000000 + 16 * 4 * 8 - 8) == pks.PKS_E_ARG


def test_workspace_too_small():
    need = lib.pks_workspace_bytes(4, 2, 5000, 1, 0)
    assert call_filter(fake_model(), T=5000, ws_bytes=need - 1) == pks.PKS_E_WORKSPACE
    assert "workspace" in lib.pks_last_error().decode()


def test_smoother_argument_errors():
    m = fake_model()
    wsb = lib.pks_workspace_bytes(4, 2, 16, 1, 0)
    assert lib.pks_smooth(ctypes.byref(m), 16, FAKE, FAKE + 0x1000000, None, FAKE + 0x3000000, 0,
                          FAKE + 0x8000000, wsb, None) == pks.PKS_E_ARG
    # output overlapping the filtered input
    assert lib.pks_smooth(ctypes.byref(m), 16, FAKE, FAKE + 0x1000000, FAKE + 8, FAKE + 0x3000000, 0,
                          FAKE + 0x8000000, wsb, None) == pks.PKS_E_ARG


def test_batched_argument_errors():
    m = fake_model(per_sequence=1)
    wsb = lib.pks_workspace_bytes(4, 2, 100, 3, 0)
    args = (FAKE + 0x1000000, FAKE + 0x2000000, FAKE + 0x3000000, 0, FAKE + 0x8000000, wsb, None)
    assert lib.pks_filter_batched(ctypes.byref(m), 0, FAKE, 100, *args) == pks.PKS_E_ARG
    assert lib.pks_filter_batched(ctypes.byref(m), 3, None, 100, *args) == pks.PKS_E_ARG
    assert lib.pks_filter_batched(ctypes.byref(m), 3, FAKE, -5, *args) == pks.PKS_E_ARG


def test_check_offsets_argument_errors():
    bad = ctypes.c_int32(7)
    assert lib.pks_check_offsets(0, FAKE, 10, FAKE, ctypes.byref(bad), None) == pks.PKS_E_ARG and bad.value == -1
    assert lib.pks_check_offsets(3, None, 10, FAKE, None, None) == pks.PKS_E_ARG
    assert lib.pks_check_offsets(3, FAKE, 10, None, None, None) == pks.PKS_E_ARG
    assert lib.pks_check_offsets(3, FAKE, -1, FAKE, None, None) == pks.PKS_E_ARG


def test_plan_and_tuner_argument_errors():
    assert lib.pks_plan_destroy(None) == pks.PKS_OK
    assert lib.pks_plan_launch(None, None) == pks.PKS_E_ARG
    h = ctypes.c_void_p()
    m = fake_model()
    # offsets NULL with B != 1
    assert lib.pks_plan_create(ctypes.byref(m), 2, None, 10, FAKE, FAKE + 0x1000000, FAKE + 0x2000000,
                               FAKE + 0x3000000, FAKE + 0x4000000, 0, FAKE + 0x8000000, 1 << 30, None, None,
                               ctypes.byref(h)) == pks.PKS_E_ARG
    old = os.environ.pop("PKS_TUNE_CACHE", None)
    try:
        assert lib.pks_autotune(4, 2, 1, 1000, 0, None, None) == pks.PKS_E_ARG
    finally:
        if old is not None:
            os.environ["PKS_TUNE_CACHE"] = old
    assert lib.pks_autotune(0, 2, 1, 1000, 0, b"/tmp/x.json", None) == pks.PKS_E_ARG


def test_loglik_argument_errors():
    m = fake_model()
    wsb = lib.pks_workspace_bytes(4, 2, 16, 1, 0)
    y, mm, P, ll, tot, ws = (FAKE + 0x1000000, FAKE + 0x2000000, FAKE + 0x3000000, FAKE + 0x4000000,
                             FAKE + 0x5000000, FAKE + 0x8000000)
    call = lambda **kw: lib.pks_loglik(
        kw.get("model", ctypes.byref(m)), kw.get("T", 16), kw.get("y", y), kw.get("m", mm), kw.get("P", P),
        kw.get("ll", ll), kw.get("tot", tot), kw.get("cum", 0), kw.get("prec", 0), kw.get("ws", ws),
        kw.get("wsb", wsb), None)
    assert call(model=None) == pks.PKS_E_ARG
    assert call(ll=None, tot=None) == pks.PKS_E_ARG              # no output
    assert call(ll=None, cum=1) == pks.PKS_E_ARG                 # prefix sums need ll
    assert call(y=None) == pks.PKS_E_ARG
    assert call(P=None) == pks.PKS_E_ARG
    assert call(T=-1) == pks.PKS_E_ARG
    assert call(prec=2) == pks.PKS_E_ARG
    assert call(ws=None) == pks.PKS_E_ARG
    assert call(wsb=wsb - 1) == pks.PKS_E_WORKSPACE
    assert call(ll=y + 8) == pks.PKS_E_ARG                       # ll overlaps y
    assert call(tot=ll + 8) == pks.PKS_E_ARG                     # total overlaps ll
    assert call(model=ctypes.byref(fake_model(per_sequence=1))) == pks.PKS_E_ARG
    mb = fake_model(per_sequence=1)
    wsb3 = lib.pks_workspace_bytes(4, 2, 100, 3, 0)
    assert lib.pks_loglik_batched(ctypes.byref(mb), 0, FAKE, 100, y, mm, P, ll, tot, 0, 0, ws, wsb3,
                                  None) == pks.PKS_E_ARG
    assert lib.pks_loglik_batched(ctypes.byref(mb), 3, None, 100, y, mm, P, ll, tot, 0, 0, ws, wsb3,
                                  None) == pks.PKS_E_ARG


def test_workspace_covers_loglik_buffers():
    # two doubles per step (factors and block prefix sums) plus the block aggregates
    a = lib.pks_workspace_bytes(4, 2, 1 << 20, 1, 0)
    b = lib.pks_workspace_bytes(4, 2, 2 << 20, 1, 0)
    assert b - a >= 16 * (1 << 20)


def test_time_varying_argument_errors():
    assert lib.pks_workspace_bytes_tv(4, 2, 100, 0) > lib.pks_workspace_bytes(4, 2, 100, 1, 0)
    for bad in ((0, 2, 10, 0), (4, 65, 10, 0), (4, 2, -1, 0), (4, 2, 1 << 31, 0), (4, 2, 10, 5)):
        assert lib.pks_workspace_bytes_tv(*bad) == 0
    t = pks.pks_model_tv()
    t.nx, t.ny = 4, 2
    for i, f in enumerate(("F", "Q", "H", "R", "m0", "P0")):
        setattr(t, f, FAKE + 0x100000 * (i + 1))
    wsb = lib.pks_workspace_bytes_tv(4, 2, 16, 0)
    y, m, P, ws = FAKE + 0x1000000, FAKE + 0x2000000, FAKE + 0x3000000, FAKE + 0x8000000
    assert lib.pks_filter_tv(None, 16, y, m, P, 0, ws, wsb, None) == pks.PKS_E_ARG
    assert lib.pks_filter_tv(ctypes.byref(t), 16, y, m, P, 0, ws, wsb - 1, None) == pks.PKS_E_WORKSPACE
    assert lib.pks_filter_tv(ctypes.byref(t), 1 << 31, y, m, P, 0, ws, 1 << 40, None) == pks.PKS_E_UNSUPPORTED
    assert lib.pks_filter_tv(ctypes.byref(t), 16, y, y + 8, P, 0, ws, wsb, None) == pks.PKS_E_ARG
    assert lib.pks_smooth_tv(ctypes.byref(t), 16, m, P, None, FAKE + 0x4000000, 0, ws, wsb, None) == pks.PKS_E_ARG
    t.Q = None
    assert lib.pks_filter_smooth_tv(ctypes.byref(t), 16, y, m, P, FAKE + 0x4000000, FAKE + 0x5000000, 0, ws,
                                    wsb, None) == pks.PKS_E_ARG
    assert lib.pks_loglik_tv(ctypes.byref(t), 16, y, m, P, FAKE + 0x4000000, None, 0, 0, ws, wsb,
                             None) == pks.PKS_E_ARG


def test_time_varying_batched_argument_errors():
    t = pks.pks_model_tv()
    t.nx, t.ny = 3, 2
    for i, f in enumerate(("F", "Q", "H", "R", "m0", "P0")):
        setattr(t, f, FAKE + 0x100000 * (i + 1))
    t.per_sequence = 1
    wsb = lib.pks_workspace_bytes_tv(3, 2, 100, 0)
    y, m, P, ws = FAKE + 0x1000000, FAKE + 0x2000000, FAKE + 0x3000000, FAKE + 0x8000000
    # per-sequence priors need a batched call
    assert lib.pks_filter_tv(ctypes.byref(t), 100, y, m, P, 0, ws, wsb, None) == pks.PKS_E_ARG
    assert lib.pks_filter_tv_batched(ctypes.byref(t), 0, FAKE, 100, y, m, P, 0, ws, wsb, None) == pks.PKS_E_ARG
    assert lib.pks_filter_tv_batched(ctypes.byref(t), 3, None, 100, y, m, P, 0, ws, wsb, None) == pks.PKS_E_ARG
    assert lib.pks_filter_tv_batched(ctypes.byref(t), 3, FAKE, 100, y, m, P, 0, ws, wsb - 1,
                                     None) == pks.PKS_E_WORKSPACE
    assert lib.pks_smooth_tv_batched(ctypes.byref(t), 3, FAKE, 100, m, P, m + 8, FAKE + 0x4000000, 0, ws, wsb,
                                     None) == pks.PKS_E_ARG
    assert lib.pks_loglik_tv_batched(ctypes.byref(t), 3, FAKE, 100, y, m, P, None, None, 0, 0, ws, wsb,
                                     None) == pks.PKS_E_ARG


def test_hmm_workspace_and_argument_errors():
    """Discrete-state HMM entry points: workspace sizing and validation."""
    assert lib.pks_hmm_workspace_bytes(0, 10) == 0 and lib.pks_hmm_workspace_bytes(65, 10) == 0
    assert lib.pks_hmm_workspace_bytes(4, -1) == 0
    assert 0 < lib.pks_hmm_workspace_bytes(4, 100) < lib.pks_hmm_workspace_bytes(64, 100)
    assert 0 < lib.pks_hmm_workspace_bytes(64, 1 << 16) <= lib.pks_hmm_workspace_bytes(64, 1 << 20)
    m = pks.pks_hmm()
    m.K, m.Pi, m.p0 = 4, FAKE, FAKE + 0x1000
    need = lib.pks_hmm_workspace_bytes(4, 16)
    L, a, lp, g, ws = FAKE + 0x100000, FAKE + 0x200000, FAKE + 0x300000, FAKE + 0x400000, FAKE + 0x800000
    f = lambda mp, T=16, L=L, a=a, lp=lp, ws=ws, n=need: lib.pks_hmm_filter(mp, T, L, a, lp, ws, n, None)
    assert f(None) == pks.PKS_E_ARG
    assert f(ctypes.byref(m), T=-1) == pks.PKS_E_ARG
    assert f(ctypes.byref(m), L=None) == pks.PKS_E_ARG
    assert f(ctypes.byref(m), ws=None) == pks.PKS_E_ARG
    assert f(ctypes.byref(m), n=need - 1) == pks.PKS_E_WORKSPACE
    assert f(ctypes.byref(m), a=L + 8) == pks.PKS_E_ARG                  # output overlaps input
    assert f(ctypes.byref(m), T=0) == pks.PKS_OK                        # empty: nothing enqueued
    bad = pks.pks_hmm()
    bad.K, bad.Pi, bad.p0 = 65, FAKE, FAKE
    assert f(ctypes.byref(bad)) == pks.PKS_E_ARG
    bad.K, bad.Pi = 4, None
    assert f(ctypes.byref(bad)) == pks.PKS_E_ARG
    assert lib.pks_hmm_smooth(ctypes.byref(m), 16, a, None, ws, need, None) == pks.PKS_E_ARG
    assert lib.pks_hmm_smooth(ctypes.byref(m), 16, a, a + 8, ws, need, None) == pks.PKS_E_ARG
    assert lib.pks_hmm_filter_smooth(ctypes.byref(m), 16, L, a, lp, L, ws, need, None) == pks.PKS_E_ARG
