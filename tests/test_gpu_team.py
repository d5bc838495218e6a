"""GPU parity of the team kernels (variant 4: each chain cut into P segments, one lane each, combined by
segmented scans across lanes) against the FP64 oracle, for every segment count (needs an MI355X)."""

import os

import numpy as np
import pytest
import torch

import oracle
from paper_1609_04493_amd import api, synth

pytestmark = pytest.mark.gpu

THREADS = min(16, len(os.sched_getaffinity(0)))
TOL32 = 1e-4


def to_dev(a, device, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(device)


def rel_rows(x, ref):
    return np.linalg.norm(np.asarray(x, np.float64) - ref, axis=-1) / np.linalg.norm(ref, axis=-1)


def rel_ragged(x, ref, link_ptr):
    return np.array([np.linalg.norm(x[a:b] - ref[a:b]) / np.linalg.norm(ref[a:b])
                     for a, b in zip(link_ptr[:-1], link_ptr[1:])])


def with_team(op, P):
    api.set_launch(op, 0, 0, 4, P)


@pytest.fixture(autouse=True)
def _reset_launch():
    yield
    api._launch_override.clear()


@pytest.mark.parametrize("P", [1, 2, 4, 8, 16, 32, 64])
def test_fp64_team_id_every_segment_count(device, P):
    """FP64 inverse dynamics of a 13-link chain (ragged tail of 67 states, base motion, tip wrenches) and of
    ragged chains of 1..64 links: equal to the oracle's serial recursion to rounding."""
    print(f"case: fp64 team ID P={P}", flush=True)
    with_team(api.OP_RNEA_ID, P)
    ch = synth.make_chains([13], 41)
    st = synth.make_states((67, 13), 41)
    rng = np.random.default_rng(41)
    tip = rng.standard_normal((67, 6))
    V0, dV0 = rng.standard_normal(6), rng.standard_normal(6)
    model = api.Model(ch, device, torch.float64)
    d = lambda a: to_dev(a, device, torch.float64)
    tau = api.rnea_id(model, d(st.q), d(st.qd), d(st.qdd), base_vel=tuple(V0), base_acc=tuple(dV0),
                      tip=d(tip)).cpu().numpy()
    for s in range(67):
        ref = oracle.rnea1(ch, st.q[s], st.qd[s], st.qdd[s], V0, dV0, tip[s])
        assert np.linalg.norm(tau[s] - ref) <= 1e-12 * np.linalg.norm(ref), s
    ch = synth.make_chains([1, 2, 13, 5, 30, 64, 7] * 11, 43)
    st = synth.make_states((ch.n_links_total,), 43)
    for prepare in (True, False):
        model = api.Model(ch, device, torch.float64, prepare=prepare)
        tau = api.rnea_id(model, d(st.q), d(st.qd), d(st.qdd)).cpu().numpy()
        ref = oracle.rnea(ch, st.q, st.qd, st.qdd)
        assert rel_ragged(tau, ref, ch.link_ptr).max() <= 1e-12, prepare


@pytest.mark.parametrize("P", [4, 8, 16, 32])
def test_fp32_team_id_uneven_4096(device, P):
    """The uneven workload (4096 chains of 10..100 links, one state each): every chain against the oracle."""
    print(f"case: fp32 team ID uneven P={P}", flush=True)
    with_team(api.OP_RNEA_ID, P)
    ch, st = synth.workload_uneven()
    model = api.Model(ch, device, torch.float32)
    d = lambda a: to_dev(a, device, torch.float32)
    tau = api.rnea_id(model, d(st.q), d(st.qd), d(st.qdd)).cpu().numpy()
    cr, sr = ch.rounded(), st.rounded()
    ref = oracle.rnea(cr, sr.q, sr.qd, sr.qdd, threads=THREADS)
    e = rel_ragged(tau, ref, ch.link_ptr)
    print(f"team ID uneven P={P}: tau max {e.max():.2e} p50 {np.median(e):.2e}", flush=True)
    assert e.max() <= TOL32


@pytest.mark.parametrize("P", [2, 4, 8])
def test_fp32_team_id_32_links_full_batch(device, P):
    """A shared 32-link chain at 16384 states (the headline shape): 512 sampled states against the oracle, and
    the whole batch against the fold kernel (same arithmetic class, FP32, so close but not bitwise)."""
    print(f"case: fp32 team ID 32 links P={P}", flush=True)
    ch, st = synth.workload_32link(16384)
    model = api.Model(ch, device, torch.float32)
    d = lambda a: to_dev(a, device, torch.float32)
    q, qd, qdd = d(st.q), d(st.qd), d(st.qdd)
    with_team(api.OP_RNEA_ID, P)
    tau = api.rnea_id(model, q, qd, qdd).cpu().numpy()
    api._launch_override.clear()
    fold = api.rnea_id(model, q, qd, qdd).cpu().numpy()
    idx = np.random.default_rng(5).choice(16384, 512, replace=False)
    cr, sr = ch.rounded(), st.rounded()
    ref = oracle.rnea(cr, sr.q[idx], sr.qd[idx], sr.qdd[idx], threads=THREADS)
    assert rel_rows(tau[idx], ref).max() <= TOL32
    assert rel_rows(tau, fold).max() <= 2 * TOL32


@pytest.mark.parametrize("P", [1, 2, 4, 8, 16])
def test_fp64_team_fd_and_id_fd_every_segment_count(device, P):
    """FP64 forward dynamics and fused ID+FD with the bias forces by team scans and the serial articulated-body
    recursions beside them: ragged chains of 1..40 links (with base motion and tip wrenches) and a shared
    13-link chain (prepared and not), equal to the oracle to rounding."""
    print(f"case: fp64 team FD P={P}", flush=True)
    with_team(api.OP_ABA_FD, P)
    with_team(api.OP_ID_FD, P)
    ch = synth.make_chains([13, 1, 40, 7, 22, 3, 16, 9], 43)
    st = synth.make_states((ch.n_links_total,), 43)
    rng = np.random.default_rng(43)
    tip = rng.standard_normal((ch.n_chains, 6))
    V0, dV0 = rng.standard_normal(6), rng.standard_normal(6)
    ref_q = oracle.aba(ch, st.q, st.qd, st.tau, V0=V0, dV0=dV0, Ftip=tip)
    ref_t = oracle.rnea(ch, st.q, st.qd, st.qdd, V0=V0, dV0=dV0, Ftip=tip)
    for prepare in (True, False):
        model = api.Model(ch, device, torch.float64, prepare=prepare)
        d = lambda a: to_dev(a, device, torch.float64)
        kw = dict(base_vel=tuple(V0), base_acc=tuple(dV0), tip=d(tip))
        q1 = api.aba_fd(model, d(st.q), d(st.qd), d(st.tau), **kw).cpu().numpy()
        t2, q2 = (x.cpu().numpy() for x in api.id_fd(model, d(st.q), d(st.qd), d(st.qdd), d(st.tau), **kw))
        assert api.read_status(device) == 0
        assert rel_ragged(q1, ref_q, ch.link_ptr).max() <= 1e-11
        assert rel_ragged(q2, ref_q, ch.link_ptr).max() <= 1e-11
        assert rel_ragged(t2, ref_t, ch.link_ptr).max() <= 1e-12
    ch1 = synth.make_chains([13], 44)
    st1 = synth.make_states((67, 13), 44)
    m1 = api.Model(ch1, device, torch.float64)
    d = lambda a: to_dev(a, device, torch.float64)
    q1 = api.aba_fd(m1, d(st1.q), d(st1.qd), d(st1.tau)).cpu().numpy()
    assert rel_rows(q1, oracle.aba(ch1, st1.q, st1.qd, st1.tau)).max() <= 1e-11


@pytest.mark.parametrize("P", [4, 8, 16])
def test_fp32_team_id_fd_uneven_4096(device, P):
    """The uneven batch (4096 chains of 10..100 links, one state each), fused ID+FD by the team kernel: every
    output against the oracle (tau within 1e-4; qdd within 1e-4 up to 32 links, bounded by the conditioning of
    M above), and against the role-split kernel's outputs."""
    print(f"case: fp32 team ID+FD uneven 4096 P={P}", flush=True)
    ch, st = synth.workload_uneven()
    model = api.Model(ch, device, torch.float32)
    d = lambda a: to_dev(a, device, torch.float32)
    q, qd, qdd, tau = d(st.q), d(st.qd), d(st.qdd), d(st.tau)
    api.set_launch(api.OP_ID_FD, 0, 0, 2)
    t_ref, q_ref = (x.cpu().numpy() for x in api.id_fd(model, q, qd, qdd, tau))
    with_team(api.OP_ID_FD, P)
    t4, q4 = (x.cpu().numpy() for x in api.id_fd(model, q, qd, qdd, tau))
    assert api.read_status(device) == 0
    cr, sr = ch.rounded(), st.rounded()
    rt = oracle.rnea(cr, sr.q, sr.qd, sr.qdd, threads=THREADS)
    rq = oracle.aba(cr, sr.q, sr.qd, sr.tau, threads=THREADS)
    lens = ch.lengths()
    et, eq = rel_ragged(t4, rt, ch.link_ptr), rel_ragged(q4, rq, ch.link_ptr)
    print(f"team ID+FD P={P}: tau max {et.max():.2e}, qdd max {eq.max():.2e} (<=32 links {eq[lens <= 32].max():.2e})",
          flush=True)
    assert et.max() <= TOL32
    assert eq[lens <= 32].max() <= TOL32
    assert eq.max() <= 1e-2
    # the two kernels differ by rounding only
    assert rel_ragged(q4, q_ref.astype(np.float64), ch.link_ptr)[lens <= 32].max() <= 2 * TOL32


def test_team_id_fd_in_a_captured_graph(device):
    """The team ID+FD kernel on the uneven batch captured once in a HIP graph; every replay equals the eager call."""
    print("case: team ID+FD graph capture", flush=True)
    ch, st = synth.workload_uneven(1024, 10, 100)
    model = api.Model(ch, device, torch.float32)
    d = lambda a: to_dev(a, device, torch.float32)
    q, qd, qdd, tau = d(st.q), d(st.qd), d(st.qdd), d(st.tau)
    with_team(api.OP_ID_FD, 8)
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


def test_team_fd_segment_bound(device):
    print("case: team FD segment bound", flush=True)
    ch, st = synth.workload_uneven(64, 10, 20)
    model = api.Model(ch, device, torch.float32)
    x = to_dev(st.q, device, torch.float32)
    with_team(api.OP_ABA_FD, 32)
    with pytest.raises(api.PdynError, match="unsupported"):
        api.aba_fd(model, x, x, x)
