"""GPU forward dynamics with every recursion scanned (pdyn_aba_fd_scan) against the FP64 oracle.

FP64: every state to 1e-11 (per-state relative norm) for every segment count
from the serial phases (P = 1) to 128 lanes per state, with the bias wrench and
z-hat as one merged scan and as two (split), with base motion and a
tip wrench, on chains of 1 to 100 links and batches that leave a ragged last
workgroup. FP32 inputs (the oracle given the same rounded inputs): 2e-6. At
the 512-link, 256-state workload the default scan and the serial phases agree
at every state to 1e-10, the split form (another rounding order) to 1e-9, and
sampled states match the oracle to 1e-9.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1609_04493_amd import api, synth

pytestmark = pytest.mark.gpu

SEGMENTS = (1, 2, 4, 8, 16, 32, 64, 128)


def dev(a, device, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(device)


def state_rel(x, ref):
    return (np.linalg.norm(x - ref, axis=1) / np.linalg.norm(ref, axis=1)).max()


@pytest.mark.parametrize("n,B", [(1, 3), (5, 7), (33, 3), (100, 2)])
def test_fp64_every_segment_count(device, n, B):
    print(f"case: fp64 scanned FD {n} links x {B} states", flush=True)
    ch = synth.make_chains([n], 600 + n)
    st = synth.make_states((B, n), 600 + n)
    rng = np.random.default_rng(n)
    tip, V0, dV0 = rng.normal(size=(B, 6)), rng.normal(size=6), rng.normal(size=6)
    ref = np.stack([oracle.aba1(ch, st.q[s], st.qd[s], st.tau[s], V0, dV0, tip[s]) for s in range(B)])
    model = api.Model(ch, device, torch.float64)
    q, qd, tau, tipd = (dev(a, device, torch.float64) for a in (st.q, st.qd, st.tau, tip))
    for P in SEGMENTS:
        for split in (False, True):
            qdd = api.aba_fd_scan(model, q, qd, tau, base_vel=V0, base_acc=dV0, tip=tipd, segments=P,
                                  split=split).cpu().numpy()
            assert api.read_status(device) == 0, (P, split)
            assert state_rel(qdd, ref) <= 1e-11, (P, split)


def test_fp32_inputs(device):
    print("case: fp32 scanned FD 100 links", flush=True)
    n, B = 100, 5
    ch = synth.make_chains([n], 670)
    chr_ = synth.Chains(*(a.astype(np.float32).astype(np.float64) for a in (ch.placement, ch.twist, ch.inertia)),
                        ch.link_ptr)
    st = synth.make_states((B, n), 670).rounded()
    ref = np.stack([oracle.aba1(chr_, st.q[s], st.qd[s], st.tau[s]) for s in range(B)])
    model = api.Model(ch, device, torch.float32)
    q, qd, tau = (dev(a, device, torch.float32) for a in (st.q, st.qd, st.tau))
    for P in (1, 16, 64, 128):
        for split in (False, True):
            qdd = api.aba_fd_scan(model, q, qd, tau, segments=P, split=split).cpu().numpy().astype(np.float64)
            assert state_rel(qdd, ref) <= 2e-6, (P, split)


def test_long_chain_batch(device):
    n, B = 512, 256
    print(f"case: scanned FD {n} links x {B} states", flush=True)
    ch = synth.make_chains([n], 3)
    st = synth.make_states((B, n), 3)
    model = api.Model(ch, device, torch.float64)
    q, qd, tau = (dev(a, device, torch.float64) for a in (st.q, st.qd, st.tau))
    qs = api.aba_fd_scan(model, q, qd, tau).cpu().numpy()
    q1 = api.aba_fd_scan(model, q, qd, tau, segments=1).cpu().numpy()
    qsp = api.aba_fd_scan(model, q, qd, tau, split=True).cpu().numpy()
    assert api.read_status(device) == 0
    assert state_rel(qs, q1) <= 1e-10
    assert state_rel(qsp, qs) <= 1e-9  # another rounding order; the same bound as against the oracle below
    for s in (0, B - 1):
        ref = oracle.aba1(ch, st.q[s], st.qd[s], st.tau[s])
        assert state_rel(qs[s:s + 1], ref[None]) <= 1e-9, s


def test_empty_batch_and_pivot_status(device):
    print("case: scanned FD empty batch, non-physical tip inertia", flush=True)
    n = 6
    ch = synth.make_chains([n], 2)
    model = api.Model(ch, device, torch.float64)
    z = torch.zeros((0, n), dtype=torch.float64, device=device)
    assert api.aba_fd_scan(model, z, z, z).shape == (0, n)
    bad = synth.Chains(ch.placement, ch.twist, ch.inertia.copy(), ch.link_ptr)
    bad.inertia[n - 1] *= -1.0
    st = synth.make_states((3, n), 2)
    mb = api.Model(bad, device, torch.float64)
    q, qd, tau = (dev(a, device, torch.float64) for a in (st.q, st.qd, st.tau))
    for P in (1, 4):
        api.aba_fd_scan(mb, q, qd, tau, segments=P)
        assert api.read_status(device) & api.STATUS_PIVOT, P


def test_unprepared_tables_and_agreement_with_aba_fd(device):
    """Tables derived inside the workspace (no pdyn_model_prepare) give the same qdd bit for bit; the FP32
    scan agrees with the role-split forward dynamics (pdyn_aba_fd) at the 512-link workload."""
    n, B = 512, 64
    print(f"case: scanned FD unprepared tables, vs pdyn_aba_fd, {n} links x {B}", flush=True)
    ch = synth.make_chains([n], 4)
    st = synth.make_states((B, n), 4)
    for dt in (torch.float64, torch.float32):
        q, qd, tau = (dev(a, device, dt) for a in (st.q, st.qd, st.tau))
        a = api.aba_fd_scan(api.Model(ch, device, dt), q, qd, tau).cpu().numpy()
        b = api.aba_fd_scan(api.Model(ch, device, dt, prepare=False), q, qd, tau).cpu().numpy()
        assert api.read_status(device) == 0
        assert np.array_equal(a, b)
    ref = api.aba_fd(api.Model(ch, device, torch.float32), q, qd, tau).cpu().numpy().astype(np.float64)
    assert state_rel(a.astype(np.float64), ref) <= 1e-3
