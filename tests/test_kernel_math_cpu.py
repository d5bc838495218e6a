"""The GPU path's per-state sweeps, compiled for the host, against the oracle (CPU only).

tests/kernel_cpu/sweeps_on_cpu.hip includes the kernels' own sweeps.hpp and
runs it one state at a time; this catches arithmetic slips in the kernel code
before any GPU run. In FP64 the results must agree with the oracle to rounding;
in FP32 within the per-state relative error bound used on the GPU.
"""

import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1609_04493_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kernel_cpu", "sweeps_on_cpu.hip")
MODE_ID, MODE_FD, MODE_IDFD = 1, 2, 3
SPLIT_FD, SPLIT_IDFD = 5, 7  # the role-split passes (articulated inertia beside the Newton-Euler passes)
POSE_RING = 16  # flag: B1 and the inverse dynamics take their transforms from pass P
ABI_U_ONLY = 32  # flag: the articulated hand-off holds U_i only; B2 forms 1/D_i


@pytest.fixture(scope="module")
def cpu_lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("kcpu") / "libsweeps_cpu.so")
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    extra = os.environ.get("PDYN_HOST_BUILD_FLAGS", "").split()  # set by the sanitizer run (test_sanitized_cpu)
    subprocess.run([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-host-only", *extra, "-o", out, SRC],
                   check=True)
    lib = ctypes.CDLL(out)
    for f in (lib.cpu_dynamics_f32, lib.cpu_dynamics_f64):
        f.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p] * 13
        f.restype = ctypes.c_int
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def run_cpu(lib, mode, chains, st, dtype, tip=None, V0=None, dV0=None):
    dt = np.dtype(dtype)
    fn = lib.cpu_dynamics_f64 if dt == np.float64 else lib.cpu_dynamics_f32
    conv = lambda a: None if a is None else np.ascontiguousarray(a, dtype=dt)
    n_chains = chains.n_chains
    q = conv(st.q)
    n_states = q.shape[0] if n_chains == 1 else n_chains
    n_max = int(chains.lengths().max())
    tau_out = np.zeros_like(q)
    qdd_out = np.zeros_like(q)
    V0 = conv(np.zeros(6) if V0 is None else V0)
    dV0 = conv(oracle.GRAVITY_ACC if dV0 is None else dV0)
    lp = np.ascontiguousarray(chains.link_ptr, dtype=np.int32)
    fn(mode, n_states, n_chains, n_max, _p(lp), _p(conv(chains.placement)), _p(conv(chains.twist)),
       _p(conv(chains.inertia)), _p(q), _p(conv(st.qd)), _p(conv(st.qdd)), _p(conv(st.tau)),
       _p(tau_out), _p(qdd_out), _p(conv(tip)), _p(V0), _p(dV0))
    return tau_out, qdd_out


def rel_err_rows(x, ref):
    return np.linalg.norm(x - ref, axis=-1) / np.linalg.norm(ref, axis=-1)


def test_fp64_sweeps_match_oracle_7_links(cpu_lib):
    ch, st = synth.workload_fp64_7link(64)
    tau, qdd = run_cpu(cpu_lib, MODE_IDFD, ch, st, np.float64)
    ref_tau = oracle.rnea(ch, st.q, st.qd, st.qdd)
    ref_qdd = oracle.aba(ch, st.q, st.qd, st.tau)
    assert rel_err_rows(tau, ref_tau).max() <= 1e-12
    assert rel_err_rows(qdd, ref_qdd).max() <= 1e-11
    t1, _ = run_cpu(cpu_lib, MODE_ID, ch, st, np.float64)
    _, q1 = run_cpu(cpu_lib, MODE_FD, ch, st, np.float64)
    assert np.array_equal(t1, tau) and np.array_equal(q1, qdd)


def test_fp64_sweeps_with_base_motion_and_tip_wrench(cpu_lib):
    ch = synth.make_chains([9], 17)
    st = synth.make_states((16, 9), 17)
    rng = np.random.default_rng(17)
    tip = rng.standard_normal((16, 6))
    V0, dV0 = rng.standard_normal(6), rng.standard_normal(6)
    tau, qdd = run_cpu(cpu_lib, MODE_IDFD, ch, st, np.float64, tip, V0, dV0)
    for s in range(16):
        rt = oracle.rnea1(ch, st.q[s], st.qd[s], st.qdd[s], V0, dV0, tip[s])
        rq = oracle.aba1(ch, st.q[s], st.qd[s], st.tau[s], V0, dV0, tip[s])
        assert np.linalg.norm(tau[s] - rt) <= 1e-12 * np.linalg.norm(rt)
        assert np.linalg.norm(qdd[s] - rq) <= 1e-11 * np.linalg.norm(rq)


def test_fp64_sweeps_ragged_chains(cpu_lib):
    ch = synth.make_chains([1, 2, 13, 5, 30], 23)
    st = synth.make_states((ch.n_links_total,), 23)
    tau, qdd = run_cpu(cpu_lib, MODE_IDFD, ch, st, np.float64)
    ref_tau = oracle.rnea(ch, st.q, st.qd, st.qdd)
    ref_qdd = oracle.aba(ch, st.q, st.qd, st.tau)
    for c in range(ch.n_chains):
        a, b = ch.link_ptr[c], ch.link_ptr[c + 1]
        assert np.linalg.norm(tau[a:b] - ref_tau[a:b]) <= 1e-12 * np.linalg.norm(ref_tau[a:b])
        assert np.linalg.norm(qdd[a:b] - ref_qdd[a:b]) <= 1e-10 * np.linalg.norm(ref_qdd[a:b])


def test_fp32_sweeps_32_links(cpu_lib):
    ch, st = synth.workload_32link(256)
    ch32, st32 = ch.astype(np.float32), st.astype(np.float32)
    tau, qdd = run_cpu(cpu_lib, MODE_IDFD, ch32, st32, np.float32)
    chr_, str_ = ch.rounded(), st.rounded()
    ref_tau = oracle.rnea(chr_, str_.q, str_.qd, str_.qdd)
    ref_qdd = oracle.aba(chr_, str_.q, str_.qd, str_.tau)
    assert rel_err_rows(tau, ref_tau).max() <= 1e-4
    assert rel_err_rows(qdd, ref_qdd).max() <= 1e-4


def test_role_split_passes_match_oracle(cpu_lib):
    """The role-split passes: FP64 to rounding (with boundary terms, ragged chains), FP32 at 32 links."""
    ch = synth.make_chains([9], 17)
    st = synth.make_states((16, 9), 17)
    rng = np.random.default_rng(17)
    tip = rng.standard_normal((16, 6))
    V0, dV0 = rng.standard_normal(6), rng.standard_normal(6)
    tau, qdd = run_cpu(cpu_lib, SPLIT_IDFD, ch, st, np.float64, tip, V0, dV0)
    _, qdd_fd = run_cpu(cpu_lib, SPLIT_FD, ch, st, np.float64, tip, V0, dV0)
    assert np.array_equal(qdd, qdd_fd)
    # transforms formed once by passes P and handed to the other passes: tau the same bits; qdd the same up to
    # rounding, since with the rings pass C takes U_i / D_i (folded by B2) instead of dividing by D_i itself
    for mode in (SPLIT_FD, SPLIT_IDFD):
        t2, q2 = run_cpu(cpu_lib, mode | POSE_RING, ch, st, np.float64, tip, V0, dV0)
        assert np.abs(q2 - qdd).max() <= 1e-12 * np.abs(qdd).max()
        if mode == SPLIT_IDFD:
            assert np.array_equal(t2, tau)
        # U_i alone handed over (1/D_i formed again by B2): the same up to rounding
        _, q3 = run_cpu(cpu_lib, mode | POSE_RING | ABI_U_ONLY, ch, st, np.float64, tip, V0, dV0)
        assert np.abs(q3 - qdd).max() <= 1e-12 * np.abs(qdd).max()
    for s in range(16):
        rt = oracle.rnea1(ch, st.q[s], st.qd[s], st.qdd[s], V0, dV0, tip[s])
        rq = oracle.aba1(ch, st.q[s], st.qd[s], st.tau[s], V0, dV0, tip[s])
        assert np.linalg.norm(tau[s] - rt) <= 1e-12 * np.linalg.norm(rt)
        assert np.linalg.norm(qdd[s] - rq) <= 1e-11 * np.linalg.norm(rq)
    ch = synth.make_chains([1, 2, 13, 5, 30], 23)
    st = synth.make_states((ch.n_links_total,), 23)
    _, qdd = run_cpu(cpu_lib, SPLIT_FD, ch, st, np.float64)
    ref = oracle.aba(ch, st.q, st.qd, st.tau)
    for c in range(ch.n_chains):
        a, b = ch.link_ptr[c], ch.link_ptr[c + 1]
        assert np.linalg.norm(qdd[a:b] - ref[a:b]) <= 1e-10 * np.linalg.norm(ref[a:b])
    _, q2 = run_cpu(cpu_lib, SPLIT_FD | POSE_RING, ch, st, np.float64)
    for c in range(ch.n_chains):
        a, b = ch.link_ptr[c], ch.link_ptr[c + 1]
        assert np.linalg.norm(q2[a:b] - qdd[a:b]) <= 1e-12 * np.linalg.norm(qdd[a:b])
    ch, st = synth.workload_32link(256)
    _, q2 = run_cpu(cpu_lib, SPLIT_FD | POSE_RING, ch.astype(np.float32), st.astype(np.float32), np.float32)
    _, q3 = run_cpu(cpu_lib, SPLIT_FD | ABI_U_ONLY, ch.astype(np.float32), st.astype(np.float32), np.float32)
    assert rel_err_rows(q3, oracle.aba(ch.rounded(), st.rounded().q, st.rounded().qd, st.rounded().tau)).max() <= 1e-4
    tau, qdd = run_cpu(cpu_lib, SPLIT_IDFD, ch.astype(np.float32), st.astype(np.float32), np.float32)
    cr, sr = ch.rounded(), st.rounded()
    assert rel_err_rows(q2, oracle.aba(cr, sr.q, sr.qd, sr.tau)).max() <= 1e-4
    e = rel_err_rows(qdd, oracle.aba(cr, sr.q, sr.qd, sr.tau))
    print(f"split fp32 qdd max rel err {e.max():.2e}")
    assert e.max() <= 1e-4
    assert rel_err_rows(tau, oracle.rnea(cr, sr.q, sr.qd, sr.qdd)).max() <= 1e-4


# ---- adjoints -----------------------------------------------------------------------

def run_vjp_cpu(lib, op, chains, q, qd, qdd, bar, dtype):
    dt = np.dtype(dtype)
    fn = lib.cpu_vjp_f64 if dt == np.float64 else lib.cpu_vjp_f32
    fn.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p] * 16
    conv = lambda a: np.ascontiguousarray(a, dtype=dt)
    n_chains = chains.n_chains
    q = conv(q)
    n_states = q.shape[0] if n_chains == 1 else n_chains
    n_max = int(chains.lengths().max())
    outs = [np.zeros_like(q) for _ in range(4)]
    pib = np.zeros((n_max if n_chains == 1 else chains.n_links_total, 10))
    lp = np.ascontiguousarray(chains.link_ptr, dtype=np.int32)
    fn(op, n_states, n_chains, n_max, _p(lp), _p(conv(chains.placement)), _p(conv(chains.twist)),
       _p(conv(chains.inertia)), _p(q), _p(conv(qd)), _p(conv(qdd)), _p(conv(bar)), *[_p(o) for o in outs],
       _p(pib), None, _p(conv(np.zeros(6))), _p(conv(oracle.GRAVITY_ACC)))
    return outs, pib


def test_fp64_adjoint_sweeps_match_oracle(cpu_lib):
    from oracle import grad
    ch = synth.make_chains([8], 41)
    st = synth.make_states((5, 8), 41)
    bar = np.random.default_rng(41).standard_normal((5, 8))
    (qb, qdb, qddb, _), pib = run_vjp_cpu(cpu_lib, 0, ch, st.q, st.qd, st.qdd, bar, np.float64)
    ref_pi = np.zeros((8, 10))
    for s in range(5):
        r = grad.rnea_vjp(ch, st.q[s], st.qd[s], st.qdd[s], bar[s])
        for x, y in zip((qb[s], qdb[s], qddb[s]), r[:3]):
            assert np.linalg.norm(x - y) <= 1e-12 * np.linalg.norm(y)
        ref_pi += r[3]
    assert np.linalg.norm(pib - ref_pi) <= 1e-12 * np.linalg.norm(ref_pi)
    qdd = oracle.aba(ch, st.q, st.qd, st.tau)
    (qb, qdb, _, tb), pib = run_vjp_cpu(cpu_lib, 1, ch, st.q, st.qd, qdd, bar, np.float64)
    ref_pi = np.zeros((8, 10))
    for s in range(5):
        r = grad.aba_vjp(ch, st.q[s], st.qd[s], st.tau[s], bar[s])
        for x, y in zip((qb[s], qdb[s], tb[s]), r[:3]):
            assert np.linalg.norm(x - y) <= 1e-11 * np.linalg.norm(y)
        ref_pi += r[3]
    assert np.linalg.norm(pib - ref_pi) <= 1e-11 * np.linalg.norm(ref_pi)


def test_role_split_adjoint_passes_match_the_fused_adjoints(cpu_lib):
    """The role-split adjoint passes equal the one-lane adjoints to rounding (FP64, boundary terms, ragged
    chains) and match the oracle's vector-Jacobian products."""
    from oracle import grad
    ch = synth.make_chains([1, 7, 12], 45)
    st = synth.make_states((ch.n_links_total,), 45)
    bar = np.random.default_rng(45).standard_normal(ch.n_links_total)
    qdd_fd = oracle.aba(ch, st.q, st.qd, st.tau)
    for op_fused, op_split, qdd in ((0, 2, st.qdd), (1, 3, qdd_fd)):
        a, pa = run_vjp_cpu(cpu_lib, op_fused, ch, st.q, st.qd, qdd, bar, np.float64)
        b, pb = run_vjp_cpu(cpu_lib, op_split, ch, st.q, st.qd, qdd, bar, np.float64)
        for x, y in zip(a, b):
            assert np.abs(x - y).max() <= 1e-11 * (np.abs(x).max() + 1e-300)
        assert np.abs(pa - pb).max() <= 1e-11 * np.abs(pa).max()
    # the ID adjoint with the overlapped kernel's hand-offs gives the same bits as the role split
    a, pa = run_vjp_cpu(cpu_lib, 2, ch, st.q, st.qd, st.qdd, bar, np.float64)
    b, pb = run_vjp_cpu(cpu_lib, 4, ch, st.q, st.qd, st.qdd, bar, np.float64)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    assert np.array_equal(pa, pb)
    # the adjoint sweep cut into a recursion and a pointwise half (with the inertia cotangents): the same bits
    for op_split, op_cut, qdd in ((2, 6, st.qdd), (3, 7, qdd_fd)):
        a, pa = run_vjp_cpu(cpu_lib, op_split, ch, st.q, st.qd, qdd, bar, np.float64)
        b, pb = run_vjp_cpu(cpu_lib, op_cut, ch, st.q, st.qd, qdd, bar, np.float64)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        assert np.array_equal(pa, pb)
    # the FD adjoint with the articulated-body pass on a third wavefront: the same bits
    a, pa = run_vjp_cpu(cpu_lib, 3, ch, st.q, st.qd, qdd_fd, bar, np.float64)
    b, pb = run_vjp_cpu(cpu_lib, 5, ch, st.q, st.qd, qdd_fd, bar, np.float64)
    for k in (0, 1, 3):
        assert np.array_equal(a[k], b[k])
    assert np.array_equal(pa, pb)
    (qb, qdb, _, tb), pib = run_vjp_cpu(cpu_lib, 3, ch, st.q, st.qd, qdd_fd, bar, np.float64)
    for c in range(ch.n_chains):
        lo, hi = ch.link_ptr[c], ch.link_ptr[c + 1]
        r = grad.aba_vjp(ch.chain(c), st.q[lo:hi], st.qd[lo:hi], st.tau[lo:hi], bar[lo:hi])
        for x, y in zip((qb[lo:hi], qdb[lo:hi], tb[lo:hi], pib[lo:hi]), r):
            assert np.linalg.norm(x - y) <= 1e-11 * np.linalg.norm(y) + 1e-14


def test_fp64_adjoint_sweeps_ragged(cpu_lib):
    from oracle import grad
    ch = synth.make_chains([2, 9, 1], 43)
    st = synth.make_states((ch.n_links_total,), 43)
    bar = np.random.default_rng(43).standard_normal(ch.n_links_total)
    (qb, qdb, qddb, _), pib = run_vjp_cpu(cpu_lib, 0, ch, st.q, st.qd, st.qdd, bar, np.float64)
    for c in range(ch.n_chains):
        a, b = ch.link_ptr[c], ch.link_ptr[c + 1]
        r = grad.rnea_vjp(ch.chain(c), st.q[a:b], st.qd[a:b], st.qdd[a:b], bar[a:b])
        for x, y in zip((qb[a:b], qdb[a:b], qddb[a:b], pib[a:b]), r):
            # (a one-link chain's qd_bar is exactly zero: absolute floor for rounding noise)
            assert np.linalg.norm(x - y) <= 1e-12 * np.linalg.norm(y) + 1e-14


def test_fp32_adjoint_sweeps_32_links(cpu_lib):
    from oracle import grad
    ch, st = synth.workload_32link(6)
    cr, sr = ch.rounded(), st.rounded()
    bar = np.random.default_rng(44).standard_normal((6, 32)).astype(np.float32).astype(np.float64)
    (qb, qdb, qddb, _), pib = run_vjp_cpu(cpu_lib, 0, cr, sr.q, sr.qd, sr.qdd, bar, np.float32)
    for s in range(6):
        r = grad.rnea_vjp(cr, sr.q[s], sr.qd[s], sr.qdd[s], bar[s])
        for x, y in zip((qb[s], qdb[s], qddb[s]), r[:3]):
            assert np.linalg.norm(x - y) <= 1e-4 * np.linalg.norm(y)


# ---- rollouts -----------------------------------------------------------------------

def test_fp64_rollout_sweeps_match_oracle(cpu_lib):
    """Forward rollout and its checkpointed adjoint (partial last segment) against the oracle."""
    from oracle import grad
    f = cpu_lib.cpu_rollout_f64
    f.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p] * 3 + [ctypes.c_int, ctypes.c_double, ctypes.c_int] + [ctypes.c_void_p] * 13
    n, B, T, dt, k = 5, 3, 23, 1e-2, 10
    ch = synth.make_chains([n], 3)
    st = synth.make_states((B, n), 3)
    tau = 10 * np.random.default_rng(1).standard_normal((T, B, n))
    C = (T + k - 1) // k
    q, qd = st.q.copy(), st.qd.copy()
    ckq, ckqd = np.zeros((C, B, n)), np.zeros((C, B, n))
    args = [_p(np.ascontiguousarray(a)) for a in (ch.placement, ch.twist, ch.inertia)]
    z6, g6 = np.zeros(6), np.ascontiguousarray(oracle.GRAVITY_ACC)
    f(0, B, n, *args, T, dt, k, _p(tau), _p(q), _p(qd), _p(ckq), _p(ckqd), None, None, None, None, None, None, _p(z6), _p(g6))
    qT_bar, qdT_bar = 2 * q, np.zeros((B, n))
    q0b, qd0b, tb, pb = np.zeros((B, n)), np.zeros((B, n)), np.zeros((T, B, n)), np.zeros((n, 10))
    f(1, B, n, *args, T, dt, k, _p(tau), None, None, _p(ckq), _p(ckqd), _p(qT_bar), _p(qdT_bar), _p(q0b), _p(qd0b),
      _p(tb), _p(pb), _p(z6), _p(g6))
    pref = np.zeros((n, 10))
    for s in range(B):
        rq, rqd = oracle.rollout1(ch, T, dt, st.q[s], st.qd[s], tau[:, s, :])
        assert np.linalg.norm(q[s] - rq) <= 1e-13 * np.linalg.norm(rq)
        assert np.array_equal(ckq[0, s], st.q[s])
        gq, gqd, gt, gpi = grad.rollout_gradient(ch, T, dt, st.q[s], st.qd[s], tau[:, s, :])
        assert np.linalg.norm(q0b[s] - gq) <= 1e-12 * np.linalg.norm(gq)
        assert np.linalg.norm(qd0b[s] - gqd) <= 1e-12 * np.linalg.norm(gqd)
        assert np.linalg.norm(tb[:, s, :] - gt) <= 1e-12 * np.linalg.norm(gt)
        pref += gpi
    assert np.linalg.norm(pb - pref) <= 1e-12 * np.linalg.norm(pref)



def test_interleaved_record_reader(cpu_lib):
    """One chain per state: a wavefront's link records interleaved over its 64 lanes in 16-byte pieces (word w
    of record i of lane l at i*32*64 + (w // V)*64*V + l*V + w % V, V = 16 / itemsize) read back exactly."""
    rng = np.random.default_rng(3)
    for dt, fn in ((np.float32, cpu_lib.cpu_read_ilv_f32), (np.float64, cpu_lib.cpu_read_ilv_f64)):
        fn.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        fn.restype = None
        n, V = 5, 16 // np.dtype(dt).itemsize
        rec = rng.standard_normal((n, 64, 32)).astype(dt)  # [record][lane][word]
        ilv = np.zeros(n * 32 * 64, dt)
        for i in range(n):
            for l in range(64):
                for w in range(32):
                    ilv[i * 32 * 64 + (w // V) * 64 * V + l * V + w % V] = rec[i, l, w]
        out = np.zeros(32, dt)
        for i, l in ((0, 0), (2, 17), (4, 63), (3, 40)):
            fn(_p(ilv), l, i, _p(out))
            assert np.array_equal(out, rec[i, l]), (dt, i, l)


def test_bounded_wait_reports_a_give_up(cpu_lib):
    """The wavefront hand-off wait of the role-split kernels: a wait that is satisfied leaves the status word
    alone; one that reaches its spin bound ORs PDYN_STATUS_WAIT (4) into it and returns the value it last read."""
    fn = cpu_lib.cpu_bounded_wait
    fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint32),
                   ctypes.POINTER(ctypes.c_int)]
    fn.restype = ctypes.c_int
    st, polls = ctypes.c_uint32(1), ctypes.c_int(0)
    assert fn(5, 7, 3, 100, ctypes.byref(st), ctypes.byref(polls)) == 7
    assert st.value == 1 and polls.value == 4  # satisfied on the 4th poll; the other bits are kept
    assert fn(5, 7, -1, 50, ctypes.byref(st), ctypes.byref(polls)) == 0
    assert st.value == 1 | 4 and polls.value == 51  # gave up after the first poll and 50 more
    st.value = 0
    assert fn(5, 4, 0, 10, ctypes.byref(st), ctypes.byref(polls)) == 4  # progress stalls below k
    assert st.value == 4
    st.value = 0
    assert fn(0, 0, -1, 10, ctypes.byref(st), ctypes.byref(polls)) == 0 and st.value == 0  # nothing to wait for
    assert polls.value == 1
    from paper_1609_04493_amd import api
    assert api.STATUS_WAIT == 4
