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
    b.max_blocks, b.variant = 0, 5  # no such kernel variant
    assert _call_id(m, b, (p, p, p, p)) == -1
    b.variant, b.segments = 4, 3  # segments must be a power of two
    assert _call_id(m, b, (p, p, p, p)) == -1
    b.segments = 128
    assert _call_id(m, b, (p, p, p, p)) == -1
    b.variant, b.segments = 0, 0
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


def _chain_model(lp_host, order_host=None, n_links_max=None, with_order=False):
    """A two-or-more-chain model whose device pointers are host addresses: only host-side checks may touch it."""
    lp_host = np.ascontiguousarray(lp_host, np.int32)
    n_chains = len(lp_host) - 1
    L = int(max(lp_host[-1], 1))
    nmax = n_links_max if n_links_max is not None else int(max(np.diff(lp_host).max(), 1))
    arrays = [np.zeros((L, k), np.float32) for k in (7, 6, 10)]
    dev_lp = lp_host.copy()
    order = None if order_host is None else np.ascontiguousarray(order_host, np.int32)
    m = api._Model(n_chains, nmax, L, dev_lp.ctypes.data, *(a.ctypes.data for a in arrays), 0,
                   0 if not with_order else order.ctypes.data,
                   lp_host.ctypes.data, 0 if order is None else order.ctypes.data)
    return m, (lp_host, dev_lp, order, arrays)


def _csr_accepted(m):
    """Host validation of a one-chain-per-state model, without launching anything: the workspace query
    returns 0 exactly when the model/batch checks fail, and pdyn_model_prepare fails before any launch."""
    L = api.lib()
    b = api._batch_struct(m.n_chains, api.ZERO6, api.GRAVITY_ACC, None)
    return L.pdyn_workspace_bytes(2, ctypes.byref(m), ctypes.byref(b), 4) > 0


def test_bad_csr_is_rejected_on_the_host():
    L = api.lib()
    good, keep = _chain_model([0, 3, 5, 9])
    assert _csr_accepted(good)
    cases = {
        "first offset not 0": [1, 3, 5, 9],
        "empty chain": [0, 3, 3, 9],
        "decreasing offsets": [0, 5, 3, 9],
        "last offset is not n_links_total": [0, 3, 5, 8],
    }
    for what, lp in cases.items():
        m, k = _chain_model(lp, n_links_max=4)
        m.n_links_total = 9
        assert not _csr_accepted(m), what
    # a chain longer than n_links_max
    m, k = _chain_model([0, 3, 5, 9], n_links_max=3)
    assert not _csr_accepted(m)
    # the host copy is required
    m, k = _chain_model([0, 3, 5, 9])
    m.link_ptr_host = 0
    assert not _csr_accepted(m)
    # the same checks guard pdyn_model_prepare and the operations themselves, before any launch
    m, k = _chain_model([0, 3, 3, 9], n_links_max=4)
    m.n_links_total = 9
    buf = np.zeros(1 << 22, np.uint8)
    p = buf.ctypes.data + ((-buf.ctypes.data) % 256)
    assert L.pdyn_model_prepare(ctypes.byref(m), 4, p, (1 << 22) - 256, None) == -1
    x = np.zeros(9, np.float32)
    b = api._batch_struct(3, api.ZERO6, api.GRAVITY_ACC, None)
    px = x.ctypes.data
    assert L.pdyn_rnea_id(ctypes.byref(m), ctypes.byref(b), px, px, px, px, p, (1 << 22) - 256, None) == -1
    assert L.pdyn_aba_fd_vjp(ctypes.byref(m), ctypes.byref(b), px, px, px, px, px, px, px, 0, p,
                             (1 << 22) - 256, None) == -1


def test_bad_order_is_rejected_on_the_host():
    good, keep = _chain_model([0, 3, 5, 9], order_host=[2, 0, 1], with_order=True)
    assert _csr_accepted(good)
    for what, order in {"duplicate": [0, 0, 1], "out of range": [0, 1, 3], "negative": [-1, 0, 1]}.items():
        m, k = _chain_model([0, 3, 5, 9], order_host=order, with_order=True)
        assert not _csr_accepted(m), what
    # a device order without its host copy
    m, k = _chain_model([0, 3, 5, 9], order_host=[2, 0, 1], with_order=True)
    m.order_host = 0
    assert not _csr_accepted(m)


def test_prepared_model_skips_the_per_call_csr_check():
    """With prepared tables the per-call check reads no host CSR (the tables carry the clamped lane map)."""
    m, keep = _chain_model([0, 3, 5, 9])
    m.link_ptr_host = 0
    assert not _csr_accepted(m)
    m.prepared = 256  # any aligned non-null pointer: only the workspace size is queried
    assert _csr_accepted(m)


def test_euler_step_validation():
    """pdyn_euler_step / _vjp: argument checks on the host, before any launch; n == 0 queues nothing."""
    L = api.lib()
    x = np.zeros(8, np.float32)
    p = x.ctypes.data
    assert L.pdyn_euler_step(0, 1e-3, p, p, p, None) == 0
    assert L.pdyn_euler_step(-1, 1e-3, p, p, p, None) == -1
    assert L.pdyn_euler_step(8, float("nan"), p, p, p, None) == -1
    assert L.pdyn_euler_step(8, 1e-3, p, None, p, None) == -1
    assert L.pdyn_euler_step(8, 1e-3, p, p + 2, p, None) == -2
    f = L.pdyn_euler_step_vjp
    assert f(0, 1e-3, p, p, None, None, None, 0, None, None, None) == 0
    assert f(8, 1e-3, p, p, p, None, p, 0, None, None, None) == -1   # q_bar_fd without qd_bar_fd
    assert f(8, 1e-3, p, p, None, None, p, 10, None, p, None) == -1  # pi_bar_fd without pi_bar
    assert f(8, 1e-3, None, p, None, None, p, 0, None, None, None) == -1
    assert f(8, 1e-3, p, p, None, None, p + 1, 0, None, None, None) == -2
    assert f(-2, 1e-3, p, p, None, None, p, 0, None, None, None) == -1


def test_load_tuning_parses_and_rejects():
    """pdyn_load_tuning: the autotuner's table form is accepted; malformed text or out-of-range values are
    rejected (PDYN_EINVAL) without replacing the installed table; NULL clears it."""
    L = api.lib()
    good = (b'{"entries": [{"op": 2, "scalar": 4, "shared": 0, "n_max": 100, "n_states": 4096, '
            b'"block": 0, "max_blocks": 0, "variant": 2},\n {"op": 0, "scalar": 8, "shared": 1, "n_max": 7, '
            b'"n_states": 64, "block": 128, "max_blocks": 256, "variant": 1}]}')
    assert L.pdyn_load_tuning(good) == 0
    assert L.pdyn_load_tuning(b'{"entries": []}') == 0
    bad = [b'{"entries": [{"op": 9, "scalar": 4, "shared": 0, "n_max": 1, "n_states": 1}]}',
           b'{"entries": [{"op": 0, "scalar": 2, "shared": 0, "n_max": 1, "n_states": 1}]}',
           b'{"entries": [{"op": 0, "scalar": 4, "shared": 0, "n_max": 1, "n_states": 1, "block": 100}]}',
           b'{"entries": [{"op": 0, "scalar": 4, "shared": 0, "n_max": 1, "n_states": 1, "variant": 7}]}',
           b'{"entries": [{"op": 0, "scalar": 4, "shared": 0, "n_max": 0, "n_states": 1}]}',
           b'{"entries": [{"op": 0, "scalar": 4, "shared": 0, "n_max": 1, "n_states": 1, "colour": 3}]}',
           b'{"entries": [{"op": 0, "scalar": 4}', b'{"rows": []}', b'{"entries": []} trailing', b'[]']
    for text in bad:
        assert L.pdyn_load_tuning(text) == -1, text
    assert L.pdyn_load_tuning(None) == 0
    assert L.pdyn_load_tuning(b"") == 0


def test_tuning_table_decides_the_launch():
    """After pdyn_load_tuning, a call that leaves its launch fields at 0 takes the nearest entry of its
    operation, precision and model kind within a factor of 2 in links and states (pdyn_launch_choice)."""
    L = api.lib()
    m, keep = _fake_model(n=32)

    def choice(op, n_states, scalar=4, fields=(0, 0, 0)):
        b = api._batch_struct(n_states, api.ZERO6, api.GRAVITY_ACC, None)
        b.block_threads, b.max_blocks, b.variant = fields
        out = [ctypes.c_int32(-9) for _ in range(4)]
        assert L.pdyn_launch_choice(op, ctypes.byref(m), ctypes.byref(b), scalar, *map(ctypes.byref, out)) == 0
        assert out[3].value == 0
        return tuple(o.value for o in out[:3])

    text = (b'{"entries": [{"op": 2, "scalar": 4, "shared": 1, "n_max": 32, "n_states": 16384, "block": 0, '
            b'"max_blocks": 0, "variant": 1}, {"op": 2, "scalar": 4, "shared": 1, "n_max": 32, "n_states": 1024, '
            b'"block": 128, "max_blocks": 64, "variant": 3}, {"op": 1, "scalar": 8, "shared": 1, "n_max": 40, '
            b'"n_states": 100, "block": 64, "max_blocks": 0, "variant": 2}]}')
    try:
        assert choice(2, 16384) == (0, 0, 0)  # no table yet: library defaults
        assert L.pdyn_load_tuning(text) == 0
        assert choice(2, 20000) == (0, 0, 1)
        assert choice(2, 1500) == (128, 64, 3)
        assert choice(2, 100) == (0, 0, 0)  # no entry within a factor of 2 in states
        assert choice(2, 16384, scalar=8) == (0, 0, 0)  # other precision
        assert choice(0, 16384) == (0, 0, 0)  # other operation
        assert choice(1, 100, scalar=8) == (64, 0, 2)  # 32 vs 40 links: within a factor of 2
        assert choice(2, 16384, fields=(64, 0, 0)) == (64, 0, 0)  # explicit launch fields win
    finally:
        assert L.pdyn_load_tuning(None) == 0
    assert choice(2, 20000) == (0, 0, 0)


def test_team_segments_resolve():
    """Variant 4 (segmented scans): the lane count per chain is the batch's, or by default the largest power of
    two up to 64 leaving at least 8 links per segment; its workspace holds one slot per link of a segment."""
    L = api.lib()
    for n, P in ((7, 1), (16, 2), (32, 4), (100, 8), (1000, 64)):
        m, keep = _fake_model(n=n)
        b = api._batch_struct(100, api.ZERO6, api.GRAVITY_ACC, None)
        b.variant = 4
        out = [ctypes.c_int32(-9) for _ in range(4)]
        assert L.pdyn_launch_choice(0, ctypes.byref(m), ctypes.byref(b), 4, *map(ctypes.byref, out)) == 0
        assert out[2].value == 4 and out[3].value == P, (n, out[3].value)
        b.segments = 16
        assert L.pdyn_launch_choice(0, ctypes.byref(m), ctypes.byref(b), 4, *map(ctypes.byref, out)) == 0
        assert out[3].value == 16
        ws = L.pdyn_workspace_bytes(0, ctypes.byref(m), ctypes.byref(b), 4)
        assert ws >= -(-n // 16) * 8 * 100 * 16 * 4


def test_team_fd_segments_resolve():
    """Forward dynamics and ID+FD with variant 4: at most 16 lanes per chain by default, and a workspace with
    the team slots of the bias forces (and, for ID+FD, of the inverse dynamics); the per-chain values of the
    serial passes live in LDS."""
    L = api.lib()
    for op in (1, 2):
        for n, P in ((7, 1), (32, 4), (100, 8), (1000, 16)):
            m, keep = _fake_model(n=n)
            b = api._batch_struct(100, api.ZERO6, api.GRAVITY_ACC, None)
            b.variant = 4
            out = [ctypes.c_int32(-9) for _ in range(4)]
            assert L.pdyn_launch_choice(op, ctypes.byref(m), ctypes.byref(b), 4, *map(ctypes.byref, out)) == 0
            assert out[3].value == P, (op, n, out[3].value)
            ws = L.pdyn_workspace_bytes(op, ctypes.byref(m), ctypes.byref(b), 4)
            team = -(-n // P) * 8 * 100 * P * 4
            assert ws >= (2 if op == 2 else 1) * team


def test_jsiia_host_rules():
    """The joint-space inertia entry points: shared chains only, null and misaligned pointers, workspace size."""
    L = api.lib()
    fn = L.pdyn_jsiia_fd
    fn.argtypes = [ctypes.POINTER(api._Model), ctypes.POINTER(api._Batch)] + [ctypes.c_void_p] * 5 + \
        [ctypes.c_size_t, ctypes.c_void_p]
    m, keep = _fake_model(n=6)
    b = api._batch_struct(8, api.ZERO6, api.GRAVITY_ACC, None)
    x = np.zeros(48, np.float32)
    p = x.ctypes.data
    ws = np.zeros((1 << 20) + 512, np.uint8)
    w = ws.ctypes.data + ((-ws.ctypes.data) % 256)
    need = L.pdyn_workspace_bytes(5, ctypes.byref(m), ctypes.byref(b), 4)
    assert need >= 8 * (13 * 6 + 21) * 8
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, 0, p, w, 1 << 20, None) == -1
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p + 2, p, p, w, 1 << 20, None) == -2
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, p, p, w, need - 1, None) == -3
    lp = np.array([0, 3, 6], np.int32)
    m2, keep2 = _fake_model(n=6, n_chains=2, link_ptr=lp)
    m2.n_links_max = 3
    m2.link_ptr_host = lp.ctypes.data
    b2 = api._batch_struct(2, api.ZERO6, api.GRAVITY_ACC, None)
    assert fn(ctypes.byref(m2), ctypes.byref(b2), p, p, p, p, w, 1 << 20, None) == -5


def test_jacobian_host_rules():
    """The Jacobian entry points: shared chains only, null pointers, workspace size, chunked workspace query."""
    L = api.lib()
    fn = L.pdyn_aba_fd_jacobian
    m, keep = _fake_model(n=5)
    b = api._batch_struct(100, api.ZERO6, api.GRAVITY_ACC, None)
    x = np.zeros(8, np.float32)
    p = x.ctypes.data
    need = L.pdyn_workspace_bytes(8, ctypes.byref(m), ctypes.byref(b), 4)
    vjp = L.pdyn_workspace_bytes(4, ctypes.byref(m), ctypes.byref(api._batch_struct(500, api.ZERO6,
                                                                                      api.GRAVITY_ACC, None)), 4)
    assert need >= vjp + 4 * 500 * 5 * 4 + 500 * 6 * 4  # the adjoint's workspace for 500 rows + expansions
    ws = np.zeros(need + 512, np.uint8)
    w = ws.ctypes.data + ((-ws.ctypes.data) % 256)
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, 0, p, p, p, w, need, None) == -1
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, p, p, p, p, w, need - 1, None) == -3
    lp = np.array([0, 3, 6], np.int32)
    m2, keep2 = _fake_model(n=6, n_chains=2, link_ptr=lp)
    m2.n_links_max = 3
    m2.link_ptr_host = lp.ctypes.data
    b2 = api._batch_struct(2, api.ZERO6, api.GRAVITY_ACC, None)
    assert fn(ctypes.byref(m2), ctypes.byref(b2), p, p, p, p, p, p, w, need, None) == -5
    assert L.pdyn_workspace_bytes(7, ctypes.byref(m2), ctypes.byref(b2), 4) == 0
    big = api._batch_struct(100000, api.ZERO6, api.GRAVITY_ACC, None)  # chunked: 2^17 / 5 states at a time
    unchunked = L.pdyn_workspace_bytes(4, ctypes.byref(m), ctypes.byref(api._batch_struct(
        500000, api.ZERO6, api.GRAVITY_ACC, None)), 4)  # one adjoint over all 100000 x 5 rows
    assert L.pdyn_workspace_bytes(8, ctypes.byref(m), ctypes.byref(big), 4) < unchunked // 3


def test_noalloc_rejects_before_device_work():
    """pdyn_id_fd_noalloc: invalid arguments and batches beyond its static scratch fail on the host."""
    L = api.lib()
    assert L.pdyn_id_fd_noalloc(None, None, 0, 0, 0, 0, 0, 0, None, None) == -1
    m, keep = _fake_model(n=32)
    m.prepared = 1 << 12  # any aligned value: no device work is queued on these paths
    x = np.zeros(8, np.float32)
    p = x.ctypes.data
    big = api._batch_struct(40000, api.ZERO6, api.GRAVITY_ACC, None)  # ~122 MiB of scratch > 64 MiB
    assert L.pdyn_workspace_bytes(2, ctypes.byref(m), ctypes.byref(big), 4) > (64 << 20)
    assert L.pdyn_id_fd_noalloc(ctypes.byref(m), ctypes.byref(big), p, p, p, p, p, p, None, None) == -3
    bneg = api._batch_struct(-1, api.ZERO6, api.GRAVITY_ACC, None)
    assert L.pdyn_id_fd_noalloc(ctypes.byref(m), ctypes.byref(bneg), p, p, p, p, p, p, None, None) == -1
    ok = api._batch_struct(16, api.ZERO6, api.GRAVITY_ACC, None)
    assert L.pdyn_id_fd_noalloc(ctypes.byref(m), ctypes.byref(ok), p, p, p, p, p, p, p + 1, None) == -2
    empty = api._batch_struct(0, api.ZERO6, api.GRAVITY_ACC, None)
    assert L.pdyn_id_fd_noalloc(ctypes.byref(m), ctypes.byref(empty), p, p, p, p, p, p, None, None) == 0


def test_hessian_host_rules():
    """pdyn_rnea_id_hessian: at least one block, shared chains only, workspace = status word + tables."""
    L = api.lib()
    fn = L.pdyn_rnea_id_hessian
    m, keep = _fake_model(n=5)
    b = api._batch_struct(3, api.ZERO6, api.GRAVITY_ACC, None)
    x = np.zeros(64, np.float32)
    p = x.ctypes.data
    need = L.pdyn_workspace_bytes(9, ctypes.byref(m), ctypes.byref(b), 4)
    assert need == 256 + L.pdyn_model_prepared_bytes(ctypes.byref(m), 4)
    ws = np.zeros(need + 512, np.uint8)
    w = ws.ctypes.data + ((-ws.ctypes.data) % 256)
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, p, None, None, None, None, w, need, None) == -1  # no block
    assert fn(ctypes.byref(m), ctypes.byref(b), None, p, p, p, None, None, None, w, need, None) == -1
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, p, None, p + 1, None, None, w, need, None) == -2
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, p, p, None, None, p, w, need - 1, None) == -3
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, p, p, None, None, p, None, need, None) == -1
    lp = np.array([0, 3, 6], np.int32)
    m2, keep2 = _fake_model(n=6, n_chains=2, link_ptr=lp)
    m2.n_links_max = 3
    m2.link_ptr_host = lp.ctypes.data
    b2 = api._batch_struct(2, api.ZERO6, api.GRAVITY_ACC, None)
    assert fn(ctypes.byref(m2), ctypes.byref(b2), p, p, p, p, p, p, p, w, need, None) == -5
    assert L.pdyn_workspace_bytes(9, ctypes.byref(m2), ctypes.byref(b2), 4) == 0
    empty = api._batch_struct(0, api.ZERO6, api.GRAVITY_ACC, None)
    assert fn(ctypes.byref(m), ctypes.byref(empty), p, p, p, p, None, None, None, w, need, None) == 0


def test_articulated_inertia_host_rules():
    """pdyn_articulated_inertia: shared chains only, segments a power of two up to 128, workspace = status word
    + tables; an empty batch queues nothing."""
    L = api.lib()
    fn = L.pdyn_articulated_inertia
    m, keep = _fake_model(n=5)
    b = api._batch_struct(3, api.ZERO6, api.GRAVITY_ACC, None)
    x = np.zeros(64, np.float32)
    p = x.ctypes.data
    need = L.pdyn_workspace_bytes(10, ctypes.byref(m), ctypes.byref(b), 4)
    assert need == 256 + L.pdyn_model_prepared_bytes(ctypes.byref(m), 4)
    ws = np.zeros(need + 512, np.uint8)
    w = ws.ctypes.data + ((-ws.ctypes.data) % 256)
    assert fn(ctypes.byref(m), ctypes.byref(b), None, p, w, need, None) == -1
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p + 1, w, need, None) == -2
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, w, need - 1, None) == -3
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, None, need, None) == -1
    for bad in (3, 256, -2):
        b.segments = bad
        assert fn(ctypes.byref(m), ctypes.byref(b), p, p, w, need, None) == -1, bad
        assert L.pdyn_workspace_bytes(10, ctypes.byref(m), ctypes.byref(b), 4) == 0
    b.segments = 128  # the scans take up to 128 lanes per state (other operations 64)
    assert L.pdyn_workspace_bytes(10, ctypes.byref(m), ctypes.byref(b), 4) == need
    assert L.pdyn_workspace_bytes(0, ctypes.byref(m), ctypes.byref(b), 4) == 0
    b.segments = 0
    lp = np.array([0, 3, 6], np.int32)
    m2, keep2 = _fake_model(n=6, n_chains=2, link_ptr=lp)
    m2.n_links_max = 3
    m2.link_ptr_host = lp.ctypes.data
    b2 = api._batch_struct(2, api.ZERO6, api.GRAVITY_ACC, None)
    assert fn(ctypes.byref(m2), ctypes.byref(b2), p, p, w, need, None) == -5
    assert L.pdyn_workspace_bytes(10, ctypes.byref(m2), ctypes.byref(b2), 4) == 0
    empty = api._batch_struct(0, api.ZERO6, api.GRAVITY_ACC, None)
    assert fn(ctypes.byref(m), ctypes.byref(empty), p, p, w, need, None) == 0


def test_aba_fd_scan_host_rules():
    """pdyn_aba_fd_scan: shared chains only; workspace = status word + tables + 26 doubles per link and state."""
    L = api.lib()
    fn = L.pdyn_aba_fd_scan
    m, keep = _fake_model(n=5)
    b = api._batch_struct(3, api.ZERO6, api.GRAVITY_ACC, None)
    x = np.zeros(64, np.float32)
    p = x.ctypes.data
    need = L.pdyn_workspace_bytes(11, ctypes.byref(m), ctypes.byref(b), 4)
    tables = L.pdyn_model_prepared_bytes(ctypes.byref(m), 4)
    assert need == 256 + (tables + 255) // 256 * 256 + (3 * 5 * 26 * 8 + 255) // 256 * 256
    ws = np.zeros(need + 512, np.uint8)
    w = ws.ctypes.data + ((-ws.ctypes.data) % 256)
    assert fn(ctypes.byref(m), ctypes.byref(b), None, p, p, p, w, need, None) == -1
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, p, p + 1, w, need, None) == -2
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, p, p, w, need - 1, None) == -3
    b.segments = 3
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, p, p, w, need, None) == -1
    b.segments, b.variant = 0, 3  # 0 / 1: the merged scan, 2: split; nothing else
    assert fn(ctypes.byref(m), ctypes.byref(b), p, p, p, p, w, need, None) == -1
    b.variant = 0
    lp = np.array([0, 3, 6], np.int32)
    m2, keep2 = _fake_model(n=6, n_chains=2, link_ptr=lp)
    m2.n_links_max = 3
    m2.link_ptr_host = lp.ctypes.data
    b2 = api._batch_struct(2, api.ZERO6, api.GRAVITY_ACC, None)
    assert fn(ctypes.byref(m2), ctypes.byref(b2), p, p, p, p, w, need, None) == -5
    assert L.pdyn_workspace_bytes(11, ctypes.byref(m2), ctypes.byref(b2), 4) == 0
    empty = api._batch_struct(0, api.ZERO6, api.GRAVITY_ACC, None)
    assert fn(ctypes.byref(m), ctypes.byref(empty), p, p, p, p, w, need, None) == 0
