"""The C ABI loads, exports what include/pdyn.h declares, and rejects bad arguments on the host (CPU only).

Only argument checks that fail before any device work are exercised here: no
kernel is launched without a GPU.
"""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1609_04493_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdyn.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdyn_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = api.lib()
    names = declared_functions()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def _fake_model(n=4, n_chains=1, link_ptr=None, aligned=True):
    pl = np.zeros((n, 7), np.float32)
    tw = np.zeros((n, 6), np.float32)
    ine = np.zeros((n, 10), np.float32)
    ptr = lambda a: a.ctypes.data + (0 if aligned else 1)
    m = api._Model(n_chains, n, n, 0 if link_ptr is None else link_ptr.ctypes.data, ptr(pl), ptr(tw), ptr(ine), 0)
    return m, (pl, tw, ine)


def _call_id(m, b, arrays, ws_bytes=1 << 20, ws_align=256):
    L = api.lib()
    ws = np.zeros(ws_bytes + 512, np.uint8)
    wptr = ws.ctypes.data + ((-ws.ctypes.data) % 256) + (ws_align % 256)
    q, qd, qdd, tau = arrays
    return L.pdyn_rnea_id(ctypes.byref(m), ctypes.byref(b), q, qd, qdd, tau, wptr, ws_bytes, None)


def test_validation_codes():
    L = api.lib()
    m, keep = _fake_model()
    b = api._batch_struct(8, api.ZERO6, api.GRAVITY_ACC, None)
    x = np.zeros((8, 4), np.float32)
    p = x.ctypes.data
    # null model / batch
    assert L.pdyn_rnea_id(None, ctypes.byref(b), p, p, p, p, p, 1 << 20, None) == -1
    assert L.pdyn_rnea_id(ctypes.byref(m), None, p, p, p, p, p, 1 << 20, None) == -1
    # null joint pointer
    assert _call_id(m, b, (p, p, 0, p)) == -1
    # misaligned joint pointer
    assert _call_id(m, b, (p, p + 1, p, p)) == -2
    # misaligned workspace
    assert _call_id(m, b, (p, p, p, p), ws_align=4) == -2
    # workspace too small
    need = L.pdyn_workspace_bytes(0, ctypes.byref(m), ctypes.byref(b), 4)
    assert need > 0
    assert _call_id(m, b, (p, p, p, p), ws_bytes=need - 1) == -3
    # negative batch, bad link counts
    bneg = api._batch_struct(-1, api.ZERO6, api.GRAVITY_ACC, None)
    assert _call_id(m, bneg, (p, p, p, p)) == -1
    m0, keep0 = _fake_model(n=4)
    m0.n_links_max = 0
    assert _call_id(m0, b, (p, p, p, p)) == -1
    # too many links
    mbig, keepb = _fake_model(n=4)
    mbig.n_links_max = mbig.n_links_total = L.pdyn_max_links() + 1
    assert _call_id(mbig, b, (p, p, p, p)) == -5
    # per-state chains: n_chains must equal n_states and link_ptr is required
    lp = np.array([0, 2, 4], np.int32)
    mc, keepc = _fake_model(n=4, n_chains=2, link_ptr=lp)
    mc.n_links_max = 2
    assert _call_id(mc, b, (p, p, p, p)) == -1
    mc.link_ptr = 0
    b2 = api._batch_struct(2, api.ZERO6, api.GRAVITY_ACC, None)
    assert _call_id(mc, b2, (p, p, p, p)) == -1
    # misaligned model arrays
    ma, keepa = _fake_model(aligned=False)
    assert _call_id(ma, b, (p, p, p, p)) == -2


def test_empty_batch_is_a_no_op():
    m, keep = _fake_model()
    b = api._batch_struct(0, api.ZERO6, api.GRAVITY_ACC, None)
    assert _call_id(m, b, (0, 0, 0, 0)) == 0


def test_workspace_query():
    L = api.lib()
    m, keep = _fake_model(n=32)
    b = api._batch_struct(1000, api.ZERO6, api.GRAVITY_ACC, None)
    w_id = L.pdyn_workspace_bytes(0, ctypes.byref(m), ctypes.byref(b), 4)
    w_fd = L.pdyn_workspace_bytes(1, ctypes.byref(m), ctypes.byref(b), 4)
    w_idfd = L.pdyn_workspace_bytes(2, ctypes.byref(m), ctypes.byref(b), 4)
    w_idfd64 = L.pdyn_workspace_bytes(2, ctypes.byref(m), ctypes.byref(b), 8)
    assert 0 < w_id < w_fd <= w_idfd < w_idfd64
    assert all(w % 256 == 0 for w in (w_id, w_fd, w_idfd))
    # scratch alone is [links][words][states] scalars
    assert w_idfd >= 32 * 12 * 1000 * 4
    assert L.pdyn_workspace_bytes(99, ctypes.byref(m), ctypes.byref(b), 4) == 0
    assert L.pdyn_workspace_bytes(0, ctypes.byref(m), ctypes.byref(b), 2) == 0
    assert L.pdyn_model_prepared_bytes(ctypes.byref(m), 4) >= 32 * 32 * (4 + 8)


def test_strerror():
    L = api.lib()
    for code in (0, -1, -2, -3, -4, -5, 17):
        assert len(L.pdyn_strerror(code)) > 0


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(api, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(api, "_lib", None)
    with pytest.raises(api.PdynError):
        api.lib()


def test_launch_shape_and_order_validation():
    L = api.lib()
    m, keep = _fake_model()
    x = np.zeros((8, 4), np.float32)
    p = x.ctypes.data
    b = api._batch_struct(8, api.ZERO6, api.GRAVITY_ACC, None)
    b.block_threads = 100  # not a multiple of 64
    assert _call_id(m, b, (p, p, p, p)) == -1
    b.block_threads = 512  # above the largest workgroup
    assert _call_id(m, b, (p, p, p, p)) == -1
    b.block_threads, b.max_blocks = 64, -3
    assert _call_id(m, b, (p, p, p, p)) == -1
    b.max_blocks, b.variant = 0, 4  # no such kernel variant
    assert _call_id(m, b, (p, p, p, p)) == -1
    order = np.arange(8, dtype=np.int32)
    m.order = order.ctypes.data  # an order with a shared chain is meaningless
    b2 = api._batch_struct(8, api.ZERO6, api.GRAVITY_ACC, None)
    assert _call_id(m, b2, (p, p, p, p)) == -1


def test_read_status_validation():
    """pdyn_read_status rejects a null workspace or result pointer and a misaligned workspace before any
    device call."""
    L = api.lib()
    bits = ctypes.c_uint32(7)
    buf = np.zeros(1024, np.uint8)
    p = buf.ctypes.data + ((-buf.ctypes.data) % 256)
    assert L.pdyn_read_status(None, None, ctypes.byref(bits)) == -1
    assert L.pdyn_read_status(ctypes.c_void_p(p), None, None) == -1
    assert L.pdyn_read_status(ctypes.c_void_p(p + 4), None, ctypes.byref(bits)) == -2
    assert bits.value == 7  # untouched on error


def test_workspace_holds_the_status_word():
    """Every workspace size includes the 256-byte status block at its start."""
    L = api.lib()
    m, keep = _fake_model(n=1)
    b = api._batch_struct(1, api.ZERO6, api.GRAVITY_ACC, None)
    for op in range(5):
        assert L.pdyn_workspace_bytes(op, ctypes.byref(m), ctypes.byref(b), 4) >= 256 + 256
