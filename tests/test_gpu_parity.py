"""GPU parity of the HIP path against the FP64 oracle (needs an MI355X).

FP64 kernels must match the oracle to rounding (1e-12 relative per state for
tau, 1e-11 for qdd). FP32 kernels are held to the per-state relative error
||x - x*|| / ||x*|| <= 1e-4 (the stated bound at 32 links); the oracle runs on
the FP32-rounded inputs promoted to FP64, so the difference is kernel
arithmetic only.
"""

import os

import numpy as np
import pytest
import torch

import oracle
from paper_1609_04493_amd import api, synth

pytestmark = pytest.mark.gpu

THREADS = min(16, len(os.sched_getaffinity(0)))
TOL32 = 1e-4


def rel_rows(x, ref):
    x = np.asarray(x, np.float64)
    return np.linalg.norm(x - ref, axis=-1) / np.linalg.norm(ref, axis=-1)


def rel_ragged(x, ref, link_ptr):
    out = np.empty(len(link_ptr) - 1)
    for c in range(len(out)):
        a, b = link_ptr[c], link_ptr[c + 1]
        out[c] = np.linalg.norm(x[a:b] - ref[a:b]) / np.linalg.norm(ref[a:b])
    return out


def to_dev(a, device, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(device)


def run_all(model, st, device, dtype, **kw):
    q, qd, qdd, tau = (to_dev(a, device, dtype) for a in (st.q, st.qd, st.qdd, st.tau))
    t1 = api.rnea_id(model, q, qd, qdd, **kw)
    q1 = api.aba_fd(model, q, qd, tau, **kw)
    t2, q2 = api.id_fd(model, q, qd, qdd, tau, **kw)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (t1, q1, t2, q2)]


def test_fp64_7_links_64_states(device):
    print("case: fp64 7 links x 64 states", flush=True)
    ch, st = synth.workload_fp64_7link(64)
    model = api.Model(ch, device, torch.float64)
    t1, q1, t2, q2 = run_all(model, st, device, torch.float64)
    ref_t = oracle.rnea(ch, st.q, st.qd, st.qdd)
    ref_q = oracle.aba(ch, st.q, st.qd, st.tau)
    assert rel_rows(t1, ref_t).max() <= 1e-12
    assert rel_rows(q1, ref_q).max() <= 1e-11
    assert rel_rows(t2, ref_t).max() <= 1e-12
    assert rel_rows(q2, ref_q).max() <= 1e-11


def test_fp64_boundary_terms_and_unprepared_model(device):
    """Base velocity and acceleration, tip wrenches, and a model without prepared tables."""
    print("case: fp64 boundary terms", flush=True)
    ch = synth.make_chains([11], 31)
    st = synth.make_states((70, 11), 31)
    rng = np.random.default_rng(31)
    tip = rng.standard_normal((70, 6))
    V0, dV0 = tuple(rng.standard_normal(6)), tuple(rng.standard_normal(6))
    model = api.Model(ch, device, torch.float64, prepare=False)
    t1, q1, t2, q2 = run_all(model, st, device, torch.float64, base_vel=V0, base_acc=dV0,
                             tip=to_dev(tip, device, torch.float64))
    for s in range(70):
        rt = oracle.rnea1(ch, st.q[s], st.qd[s], st.qdd[s], np.array(V0), np.array(dV0), tip[s])
        rq = oracle.aba1(ch, st.q[s], st.qd[s], st.tau[s], np.array(V0), np.array(dV0), tip[s])
        assert np.linalg.norm(t1[s] - rt) <= 1e-12 * np.linalg.norm(rt)
        assert np.linalg.norm(q1[s] - rq) <= 1e-11 * np.linalg.norm(rq)
        assert np.linalg.norm(t2[s] - rt) <= 1e-12 * np.linalg.norm(rt)
        assert np.linalg.norm(q2[s] - rq) <= 1e-11 * np.linalg.norm(rq)


def test_fp32_32_links_all_16384_states(device):
    """The 32-link, 16384-state workload at full size, every output checked."""
    print("case: fp32 32 links x 16384 states", flush=True)
    ch, st = synth.workload_32link(16384)
    model = api.Model(ch, device, torch.float32)
    t1, q1, t2, q2 = run_all(model, st, device, torch.float32)
    cr, sr = ch.rounded(), st.rounded()
    ref_t = oracle.rnea(cr, sr.q, sr.qd, sr.qdd, threads=THREADS)
    ref_q = oracle.aba(cr, sr.q, sr.qd, sr.tau, threads=THREADS)
    et, eq = rel_rows(t2, ref_t), rel_rows(q2, ref_q)
    print(f"tau rel err p50 {np.median(et):.2e} p99 {np.quantile(et, .99):.2e} max {et.max():.2e}; "
          f"qdd p50 {np.median(eq):.2e} p99 {np.quantile(eq, .99):.2e} max {eq.max():.2e}", flush=True)
    assert et.max() <= TOL32 and eq.max() <= TOL32
    assert rel_rows(t1, ref_t).max() <= TOL32 and rel_rows(q1, ref_q).max() <= TOL32


@pytest.mark.parametrize("B", [1, 63, 65, 200])
def test_fp32_ragged_batch_tail(device, B):
    print(f"case: fp32 tail B={B}", flush=True)
    ch = synth.make_chains([32], 7)
    st = synth.make_states((B, 32), 7)
    model = api.Model(ch, device, torch.float32)
    t1, q1, t2, q2 = run_all(model, st, device, torch.float32)
    cr, sr = ch.rounded(), st.rounded()
    assert rel_rows(t2, oracle.rnea(cr, sr.q, sr.qd, sr.qdd)).max() <= TOL32
    assert rel_rows(q2, oracle.aba(cr, sr.q, sr.qd, sr.tau)).max() <= TOL32


def test_fp32_single_link_chain(device):
    print("case: fp32 one link", flush=True)
    ch = synth.make_chains([1], 3)
    st = synth.make_states((100, 1), 3)
    model = api.Model(ch, device, torch.float32)
    t1, q1, t2, q2 = run_all(model, st, device, torch.float32)
    cr, sr = ch.rounded(), st.rounded()
    assert np.abs(t1[:, 0] - oracle.rnea(cr, sr.q, sr.qd, sr.qdd)[:, 0]).max() <= 1e-5 * np.abs(t1).max()
    assert np.abs(q1[:, 0] - oracle.aba(cr, sr.q, sr.qd, sr.tau)[:, 0]).max() <= 1e-5 * np.abs(q1).max()


def test_fp32_uneven_chains_4096(device):
    """4096 chains with 10..100 links, one state each, every output checked (error reported per length)."""
    print("case: fp32 uneven 4096 chains", flush=True)
    ch, st = synth.workload_uneven()
    model = api.Model(ch, device, torch.float32)
    t1, q1, t2, q2 = run_all(model, st, device, torch.float32)
    cr, sr = ch.rounded(), st.rounded()
    ref_t = oracle.rnea(cr, sr.q, sr.qd, sr.qdd, threads=THREADS)
    ref_q = oracle.aba(cr, sr.q, sr.qd, sr.tau, threads=THREADS)
    et, eq = rel_ragged(t2, ref_t, ch.link_ptr), rel_ragged(q2, ref_q, ch.link_ptr)
    lens = ch.lengths()
    print(f"uneven: tau max {et.max():.2e}; qdd max {eq.max():.2e}; qdd max at <=32 links "
          f"{eq[lens <= 32].max():.2e}", flush=True)
    assert et.max() <= TOL32
    assert eq[lens <= 32].max() <= TOL32
    assert eq.max() <= 1e-2  # long chains: reported, bounded by conditioning, not gated at 1e-4


def test_fp32_100_links_sampled(device):
    """100-link chain at 65536 states: 256 sampled states against the oracle."""
    print("case: fp32 100 links x 65536 sampled", flush=True)
    ch, st = synth.workload_100link_rollout(65536)
    model = api.Model(ch, device, torch.float32)
    q, qd, tau = (to_dev(a, device, torch.float32) for a in (st.q, st.qd, st.tau))
    qdd = api.aba_fd(model, q, qd, tau).cpu().numpy()
    idx = np.random.default_rng(0).choice(65536, 256, replace=False)
    cr = ch.rounded()
    sr = st.rounded()
    ref = oracle.aba(cr, sr.q[idx], sr.qd[idx], sr.tau[idx], threads=THREADS)
    e = rel_rows(qdd[idx], ref)
    print(f"100 links qdd rel err p50 {np.median(e):.2e} max {e.max():.2e}", flush=True)
    assert e.max() <= 1e-2


def test_fp32_repeat_is_bitwise_identical(device):
    ch, st = synth.workload_32link(4096)
    model = api.Model(ch, device, torch.float32)
    a = run_all(model, st, device, torch.float32)
    b = run_all(model, st, device, torch.float32)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_fp32_empty_batch(device):
    ch = synth.make_chains([5], 1)
    model = api.Model(ch, device, torch.float32)
    z = torch.zeros((0, 5), device=device)
    assert api.rnea_id(model, z, z, z).shape == (0, 5)


def test_launch_shapes_orders_and_persistence_are_bitwise_identical(device):
    """Block sizes, a persistent (capped) grid and the chain order change scheduling only, not results."""
    print("case: launch shapes", flush=True)
    ch = synth.make_chains(list(np.random.default_rng(4).integers(1, 60, 300)), 4)
    st = synth.make_states((ch.n_links_total,), 4)
    model = api.Model(ch, device, torch.float32)
    for op in (api.OP_RNEA_ID, api.OP_ABA_FD, api.OP_ID_FD):
        api.set_launch(op, 0, 0, 1)
    ref = run_all(model, st, device, torch.float32)
    for bt, cap, use_order in ((128, 0, True), (256, 1, True), (64, 2, False), (192, 0, False)):
        for op in (api.OP_RNEA_ID, api.OP_ABA_FD, api.OP_ID_FD):
            api.set_launch(op, bt, cap, 1)  # launch shapes apply to the one-wavefront variant
        model.use_order = use_order
        got = run_all(model, st, device, torch.float32)
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), (bt, cap, use_order)
    for op in (api.OP_RNEA_ID, api.OP_ABA_FD, api.OP_ID_FD):
        api.set_launch(op, 0, 0)
    model.use_order = True
    cr, sr = ch.rounded(), st.rounded()
    et = rel_ragged(ref[2], oracle.rnea(cr, sr.q, sr.qd, sr.qdd), ch.link_ptr)
    assert et.max() <= TOL32


@pytest.mark.parametrize("variant", [1, 2])
def test_per_state_tables_fp64_orders_and_preparation(device, variant):
    """One chain per state (link records interleaved over the lanes of each wavefront): FP64 with tip wrenches
    and base motion against the oracle chain by chain, and bitwise the same outputs from per-call tables, from
    prepared tables, and after the lane order changes (which lays the prepared tables out again)."""
    print(f"case: per-state tables variant {variant}", flush=True)
    for op in (api.OP_RNEA_ID, api.OP_ABA_FD, api.OP_ID_FD):
        api.set_launch(op, 0, 0, variant)
    try:
        lens = list(np.random.default_rng(12).integers(1, 40, 131))  # three wavefronts, the last one ragged
        ch = synth.make_chains(lens, 12)
        st = synth.make_states((ch.n_links_total,), 12)
        rng = np.random.default_rng(12)
        tip = rng.standard_normal((ch.n_chains, 6))
        V0, dV0 = tuple(rng.standard_normal(6)), tuple(rng.standard_normal(6))
        kw = dict(base_vel=V0, base_acc=dV0, tip=to_dev(tip, device, torch.float64))
        model = api.Model(ch, device, torch.float64)
        ref = run_all(model, st, device, torch.float64, **kw)
        lp = ch.link_ptr
        for c in range(ch.n_chains):
            a, b = lp[c], lp[c + 1]
            rt = oracle.rnea1(ch.chain(c), st.q[a:b], st.qd[a:b], st.qdd[a:b], np.array(V0), np.array(dV0), tip[c])
            rq = oracle.aba1(ch.chain(c), st.q[a:b], st.qd[a:b], st.tau[a:b], np.array(V0), np.array(dV0), tip[c])
            assert np.linalg.norm(ref[0][a:b] - rt) <= 1e-12 * np.linalg.norm(rt), c
            assert np.linalg.norm(ref[2][a:b] - rt) <= 1e-12 * np.linalg.norm(rt), c
            assert np.linalg.norm(ref[1][a:b] - rq) <= 1e-11 * np.linalg.norm(rq), c
            assert np.linalg.norm(ref[3][a:b] - rq) <= 1e-11 * np.linalg.norm(rq), c
        model.use_order = False  # prepared again for the natural order
        got = run_all(model, st, device, torch.float64, **kw)
        assert all(np.array_equal(x, y) for x, y in zip(got, ref))
        model.invalidate()  # tables derived inside each call's workspace
        for use_order in (False, True):
            model.use_order = use_order
            got = run_all(model, st, device, torch.float64, **kw)
            assert all(np.array_equal(x, y) for x, y in zip(got, ref)), use_order
    finally:
        for op in (api.OP_RNEA_ID, api.OP_ABA_FD, api.OP_ID_FD):
            api.set_launch(op, 0, 0)


def test_uneven_id_fd_in_a_captured_graph(device):
    """ID+FD of 4096 uneven chains captured once in a HIP graph; every replay equals the eager call."""
    print("case: uneven graph capture", flush=True)
    ch, st = synth.workload_uneven()
    model = api.Model(ch, device, torch.float32)
    d = lambda a: to_dev(a, device, torch.float32)
    q, qd, qdd, tau = d(st.q), d(st.qd), d(st.qdd), d(st.tau)
    out = (torch.empty_like(q), torch.empty_like(q))
    ws = api.Workspace()
    api.id_fd(model, q, qd, qdd, tau, out=out, workspace=ws)  # sizes the workspace outside capture
    eager = [x.clone() for x in out]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        api.id_fd(model, q, qd, qdd, tau, out=out, workspace=ws)
    for rep in range(3):
        out[0].fill_(float("nan"))
        out[1].fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[0], eager[0]) and torch.equal(out[1], eager[1]), f"replay {rep}"
        api.rnea_id(model, q, qd, qdd)  # eager work between replays


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_forward_dynamics_variants(device, variant):
    """The kernel variants (one wavefront per 64 states; role split; one launch per sweep) against the oracle:
    the 32-link workload at 16384 states, ragged chains, an odd batch and FP64 with boundary terms."""
    print(f"case: variant {variant}", flush=True)
    for op in (api.OP_RNEA_ID, api.OP_ABA_FD, api.OP_ID_FD):
        api.set_launch(op, 0, 0, variant)
    try:
        ch, st = synth.workload_32link(16384)
        model = api.Model(ch, device, torch.float32)
        t1, q1, t2, q2 = run_all(model, st, device, torch.float32)
        cr, sr = ch.rounded(), st.rounded()
        ref_t = oracle.rnea(cr, sr.q, sr.qd, sr.qdd, threads=THREADS)
        ref_q = oracle.aba(cr, sr.q, sr.qd, sr.tau, threads=THREADS)
        eq = rel_rows(q2, ref_q)
        print(f"variant {variant}: qdd max rel err {eq.max():.2e}", flush=True)
        assert eq.max() <= TOL32 and rel_rows(q1, ref_q).max() <= TOL32
        assert rel_rows(t2, ref_t).max() <= TOL32 and rel_rows(t1, ref_t).max() <= TOL32
        ch = synth.make_chains(list(np.random.default_rng(5).integers(1, 70, 333)), 5)
        st = synth.make_states((ch.n_links_total,), 5)
        model = api.Model(ch, device, torch.float32)
        t1, q1, t2, q2 = run_all(model, st, device, torch.float32)
        cr, sr = ch.rounded(), st.rounded()
        lens = ch.lengths()
        eq = rel_ragged(q2, oracle.aba(cr, sr.q, sr.qd, sr.tau), ch.link_ptr)
        assert eq[lens <= 32].max() <= TOL32 and eq.max() <= 1e-2
        assert np.array_equal(q1, q2)
        assert rel_ragged(t1, oracle.rnea(cr, sr.q, sr.qd, sr.qdd), ch.link_ptr).max() <= TOL32
        ch = synth.make_chains([11], 31)
        st = synth.make_states((70, 11), 31)
        rng = np.random.default_rng(31)
        tip = rng.standard_normal((70, 6))
        V0, dV0 = tuple(rng.standard_normal(6)), tuple(rng.standard_normal(6))
        model = api.Model(ch, device, torch.float64)
        t1, q1, t2, q2 = run_all(model, st, device, torch.float64, base_vel=V0, base_acc=dV0,
                                 tip=to_dev(tip, device, torch.float64))
        for s in range(70):
            rt = oracle.rnea1(ch, st.q[s], st.qd[s], st.qdd[s], np.array(V0), np.array(dV0), tip[s])
            rq = oracle.aba1(ch, st.q[s], st.qd[s], st.tau[s], np.array(V0), np.array(dV0), tip[s])
            assert np.linalg.norm(t2[s] - rt) <= 1e-12 * np.linalg.norm(rt)
            assert np.linalg.norm(t1[s] - rt) <= 1e-12 * np.linalg.norm(rt)
            assert np.linalg.norm(q1[s] - rq) <= 1e-11 * np.linalg.norm(rq)
            assert np.linalg.norm(q2[s] - rq) <= 1e-11 * np.linalg.norm(rq)
    finally:
        for op in (api.OP_RNEA_ID, api.OP_ABA_FD, api.OP_ID_FD):
            api.set_launch(op, 0, 0, 0)


def test_status_word_reports_numerical_faults(device):
    """Non-physical inertia (negative mass) sets the pivot bit, a NaN input the non-finite bit; healthy
    calls leave the word clear; reading clears it."""
    print("case: status word", flush=True)
    ch = synth.make_chains([12], 9)
    st = synth.make_states((130, 12), 9)
    d = lambda a: to_dev(a, device, torch.float32)
    ws = api.Workspace()
    model = api.Model(ch, device, torch.float32)
    q, qd, qdd, tau = d(st.q), d(st.qd), d(st.qdd), d(st.tau)
    for variant in (1, 2):
        for op in (api.OP_ABA_FD, api.OP_ID_FD, api.OP_ABA_FD_VJP, api.OP_RNEA_ID_VJP):
            api.set_launch(op, 0, 0, variant)
        api.id_fd(model, q, qd, qdd, tau, workspace=ws)
        qdd_fd = api.aba_fd(model, q, qd, tau, workspace=ws)
        api.aba_fd_vjp(model, q, qd, qdd_fd, qdd_fd, workspace=ws)
        assert ws.read_status() == 0, variant
        bad = q.clone()
        bad[7, 3] = float("nan")
        api.id_fd(model, bad, qd, qdd, tau, workspace=ws)
        assert ws.read_status() & api.STATUS_NONFINITE, variant
        assert ws.read_status() == 0  # cleared by the read
        heavy = synth.make_chains([12], 9)
        heavy.inertia[5, 0] = -3.0  # negative mass: D_i <= 0 somewhere down the chain
        m2 = api.Model(heavy, device, torch.float32)
        api.aba_fd(m2, q, qd, tau, workspace=ws)
        assert ws.read_status() & api.STATUS_PIVOT, variant
    for op in (api.OP_ABA_FD, api.OP_ID_FD, api.OP_ABA_FD_VJP, api.OP_RNEA_ID_VJP):
        api.set_launch(op, 0, 0, 0)


@pytest.mark.parametrize("n,B,dtype", [(20, 300, torch.float32), (50, 300, torch.float32), (90, 300, torch.float32),
                                        (120, 200, torch.float32), (30, 100, torch.float64)])
def test_role_split_lds_modes(device, n, B, dtype):
    """The role-split kernel's three hand-off modes, chosen by chain length: U_i in LDS with the transform
    rings (FP32 up to 61 links), U_i alone in LDS (FP32 up to ~106 links, FP64 up to ~53), and the barrier
    (longer chains). FD and ID+FD against the oracle."""
    print(f"case: lds modes n={n} B={B} {dtype}", flush=True)
    for op in (api.OP_ABA_FD, api.OP_ID_FD):
        api.set_launch(op, 0, 0, 2)
    try:
        ch = synth.make_chains([n], 60 + n)
        st = synth.make_states((B, n), 60 + n)
        model = api.Model(ch, device, dtype)
        d = lambda a: to_dev(a, device, dtype)
        q, qd, qdd, tau = d(st.q), d(st.qd), d(st.qdd), d(st.tau)
        q1 = api.aba_fd(model, q, qd, tau).cpu().numpy()
        t2, q2 = (x.cpu().numpy() for x in api.id_fd(model, q, qd, qdd, tau))
        if dtype == torch.float64:
            ref_q, ref_t = oracle.aba(ch, st.q, st.qd, st.tau), oracle.rnea(ch, st.q, st.qd, st.qdd)
            tol_q, tol_t = 1e-9, 1e-12
        else:
            cr, sr = ch.rounded(), st.rounded()
            ref_q, ref_t = oracle.aba(cr, sr.q, sr.qd, sr.tau), oracle.rnea(cr, sr.q, sr.qd, sr.qdd)
            tol_q, tol_t = (TOL32 if n <= 32 else 1e-2), TOL32
        eq = rel_rows(q1, ref_q)
        print(f"n={n}: qdd max rel err {eq.max():.2e}", flush=True)
        assert eq.max() <= tol_q and rel_rows(q2, ref_q).max() <= tol_q
        assert rel_rows(t2, ref_t).max() <= tol_t
    finally:
        for op in (api.OP_ABA_FD, api.OP_ID_FD):
            api.set_launch(op, 0, 0, 0)



def test_plan_repeats_the_call_bit_for_bit(device):
    """api.plan_id_fd marshals the arguments once; each call of the plan gives what id_fd gives."""
    print("case: id_fd plan, 32 links x 1000 states", flush=True)
    ch = synth.make_chains([32], 41)
    st = synth.make_states((1000, 32), 41)
    model = api.Model(ch, device, torch.float32)
    q, qd, qdd, tau = (torch.as_tensor(a, dtype=torch.float32).to(device) for a in (st.q, st.qd, st.qdd, st.tau))
    ref_tau, ref_qdd = api.id_fd(model, q, qd, qdd, tau)
    plan = api.plan_id_fd(model, q, qd, qdd, tau)
    for _ in range(3):
        plan.out[0].zero_()
        plan.out[1].zero_()
        plan()
        torch.cuda.synchronize()
        assert torch.equal(plan.out[0], ref_tau) and torch.equal(plan.out[1], ref_qdd)
    assert api.read_status(device) == 0
