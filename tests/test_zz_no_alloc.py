"""The allocation-free entry point pdyn_id_fd_noalloc against pdyn_id_fd (needs an MI355X).

Both run the same kernels, so their outputs must agree bit for bit; both are
also held to the FP64 oracle on sampled states (per-state relative error
<= 1e-4 at FP32). Three calls in a row share the library's static scratch:
the full 32-link x 16384-state batch, then a smaller batch of the same chain,
then a smaller per-state-chain batch without prepared tables (the derived
tables then live in the static scratch too).
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1609_04493_amd import api, synth

pytestmark = pytest.mark.gpu

TOL32 = 1e-4


def rel_rows(x, ref):
    x = np.asarray(x, np.float64)
    return np.linalg.norm(x - ref, axis=-1) / np.linalg.norm(ref, axis=-1)


def rel_ragged(x, ref, link_ptr):
    return np.array([np.linalg.norm(x[a:b] - ref[a:b]) / np.linalg.norm(ref[a:b])
                     for a, b in zip(link_ptr[:-1], link_ptr[1:])])


def dev(a, device):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).to(device)


def both(model, arrays, device):
    q, qd, qdd, tau = arrays
    t_ref, q_ref = api.id_fd(model, q, qd, qdd, tau)
    status = torch.full((1,), -1, dtype=torch.int32, device=device)
    t_na, q_na = api.id_fd_noalloc(model, q, qd, qdd, tau, status_out=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert torch.equal(t_na, t_ref) and torch.equal(q_na, q_ref)
    return t_na.cpu().numpy(), q_na.cpu().numpy()


def test_noalloc_matches_workspace_entry_point(device):
    print("case: no-alloc ID+FD, 32 links x 16384 states, then 3000 states, then 500 uneven chains", flush=True)
    ch, st = synth.workload_32link(16384)
    model = api.Model(ch, device, torch.float32)
    arrays = [dev(a, device) for a in (st.q, st.qd, st.qdd, st.tau)]
    cr, sr = ch.rounded(), st.rounded()

    # 1. the full batch (50 MiB of the 64 MiB scratch)
    t, qdd = both(model, arrays, device)
    idx = np.random.default_rng(7).choice(16384, 512, replace=False)
    ref_t = oracle.rnea(cr, sr.q[idx], sr.qd[idx], sr.qdd[idx])
    ref_q = oracle.aba(cr, sr.q[idx], sr.qd[idx], sr.tau[idx])
    assert rel_rows(t[idx], ref_t).max() <= TOL32
    assert rel_rows(qdd[idx], ref_q).max() <= TOL32

    # 2. a smaller batch of the same chain: the scratch keeps the first call's contents
    small = [a[:3000].contiguous() for a in arrays]
    t2, qdd2 = both(model, small, device)
    ref_t2 = oracle.rnea(cr, sr.q[:3000:7], sr.qd[:3000:7], sr.qdd[:3000:7])
    ref_q2 = oracle.aba(cr, sr.q[:3000:7], sr.qd[:3000:7], sr.tau[:3000:7])
    assert rel_rows(t2[::7], ref_t2).max() <= TOL32
    assert rel_rows(qdd2[::7], ref_q2).max() <= TOL32

    # 3. one chain per state, tables derived inside the static scratch
    chu, stu = synth.workload_uneven(500, 10, 100)
    mu = api.Model(chu, device, torch.float32, prepare=False)
    arr_u = [dev(a, device) for a in (stu.q, stu.qd, stu.qdd, stu.tau)]
    tu, qu = both(mu, arr_u, device)
    cur, sur = chu.rounded(), stu.rounded()
    lp = chu.link_ptr
    ref_tu = oracle.rnea(cur, sur.q, sur.qd, sur.qdd)
    ref_qu = oracle.aba(cur, sur.q, sur.qd, sur.tau)
    eq = rel_ragged(qu, ref_qu, lp)
    assert rel_ragged(tu, ref_tu, lp).max() <= TOL32
    assert eq[chu.lengths() <= 32].max() <= TOL32
    assert eq.max() <= 1e-2  # long chains: bounded by the conditioning of M(q), as in the parity tests


def test_noalloc_rejects_oversize_and_empty(device):
    print("case: no-alloc size limit and empty batch", flush=True)
    ch, _ = synth.workload_32link(4)
    model = api.Model(ch, device, torch.float32)
    big = torch.zeros((40000, 32), dtype=torch.float32, device=device)  # about 122 MiB of scratch
    with pytest.raises(api.PdynError, match="workspace"):
        api.id_fd_noalloc(model, big, big, big, big)
    empty = torch.zeros((0, 32), dtype=torch.float32, device=device)
    status = torch.full((1,), 5, dtype=torch.int32, device=device)
    api.id_fd_noalloc(model, empty, empty, empty, empty, status_out=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 5  # nothing queued for an empty batch
