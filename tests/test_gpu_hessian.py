"""GPU second derivatives of the inverse dynamics (pdyn_rnea_id_hessian) against the FP64 oracle.

The oracle takes each block by the multicomplex step; the GPU runs the
recursions of eqs. (1)-(2) on hyper-dual numbers. FP64: every entry to 1e-10
of its block's largest entry. FP32 (inputs rounded to FP32 for the oracle too):
5e-5 of the block's largest entry (the host build of the same pass measures
about 2e-6 at 32 links, the backward sweep's reversed recursion included).
At a 256-state batch of the 32-link chain, sampled states against the oracle, and for
every state two facts that hold at any size: the Christoffel identity between
the (qd, qd) and (q, qdd) blocks, and (q, qdd) = dM/dq against central
differences of the GPU mass matrix (FP64).
"""

import numpy as np
import pytest
import torch

from oracle import grad
from paper_1609_04493_amd import api, synth

pytestmark = pytest.mark.gpu

BLOCKS = api.HESSIAN_BLOCKS


def dev(a, device, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(device)


def oracle_blocks(ch, q, qd, qdd, blocks=BLOCKS, **kw):
    return {b: grad.rnea_hessian(ch, q, qd, qdd, b, **kw) for b in blocks}


def worst(H, ref):
    return max(np.abs(H[b] - ref[b]).max() / max(1.0, np.abs(ref[b]).max()) for b in ref)


@pytest.mark.parametrize("n,B", [(1, 3), (5, 4), (12, 3)])
def test_fp64_every_block_equals_oracle(device, n, B):
    print(f"case: fp64 hessian {n} links x {B} states", flush=True)
    ch = synth.make_chains([n], 90 + n)
    st = synth.make_states((B, n), 90 + n)
    model = api.Model(ch, device, torch.float64)
    q, qd, qdd = (dev(a, device, torch.float64) for a in (st.q, st.qd, st.qdd))
    H = {b: t.cpu().numpy() for b, t in api.rnea_id_hessian(model, q, qd, qdd).items()}
    assert api.read_status(device) == 0
    for s in range(B):
        ref = oracle_blocks(ch, st.q[s], st.qd[s], st.qdd[s])
        assert worst({b: H[b][s] for b in BLOCKS}, ref) <= 1e-10, s


def test_fp64_base_motion_tip_wrench_and_block_subset(device):
    print("case: fp64 hessian with base motion, tip wrench, two blocks", flush=True)
    n, B = 6, 3
    ch = synth.make_chains([n], 55)
    st = synth.make_states((B, n), 55)
    rng = np.random.default_rng(8)
    V0, dV0, tip = rng.normal(size=6), rng.normal(size=6), rng.normal(size=(B, 6))
    model = api.Model(ch, device, torch.float64)
    q, qd, qdd, tipd = (dev(a, device, torch.float64) for a in (st.q, st.qd, st.qdd, tip))
    out = {b: torch.empty((B, n, n, n), dtype=torch.float64, device=device) for b in ("q_qd", "q_qdd")}
    H = api.rnea_id_hessian(model, q, qd, qdd, blocks=("q_qd", "q_qdd"), base_vel=V0, base_acc=dV0, tip=tipd, out=out)
    assert H["q_qd"] is out["q_qd"] and set(H) == {"q_qd", "q_qdd"}
    for s in range(B):
        ref = oracle_blocks(ch, st.q[s], st.qd[s], st.qdd[s], ("q_qd", "q_qdd"), V0=V0, dV0=dV0, Ftip=tip[s])
        assert worst({b: H[b][s].cpu().numpy() for b in ref}, ref) <= 1e-10


def test_fp32_twelve_links(device):
    print("case: fp32 hessian 12 links", flush=True)
    n, B = 12, 2
    ch = synth.make_chains([n], 12)
    chr_ = synth.Chains(*(a.astype(np.float32).astype(np.float64) for a in (ch.placement, ch.twist, ch.inertia)),
                        ch.link_ptr)
    st = synth.make_states((B, n), 12).rounded()
    model = api.Model(ch, device, torch.float32)
    q, qd, qdd = (dev(a, device, torch.float32) for a in (st.q, st.qd, st.qdd))
    H = {b: t.cpu().numpy().astype(np.float64) for b, t in api.rnea_id_hessian(model, q, qd, qdd).items()}
    for s in range(B):
        ref = oracle_blocks(chr_, st.q[s], st.qd[s], st.qdd[s])
        assert worst({b: H[b][s] for b in BLOCKS}, ref) <= 5e-5


def christoffel_residual(Hvv, Hqa):
    """max |H_qdqd - (dM_ij/dq_k + dM_ik/dq_j - dM_jk/dq_i)| over states, relative to the block's scale
    (base at rest), with dM[s, a, b, c] = dM_ab / dq_c = H_qqdd[s, a, c, b]."""
    dM = np.transpose(Hqa, (0, 1, 3, 2))
    two_gamma = dM + np.transpose(dM, (0, 1, 3, 2)) - np.transpose(dM, (0, 3, 1, 2))
    return np.abs(Hvv - two_gamma).max() / np.abs(Hvv).max()


def test_full_batch_32_links(device):
    """The 32-link chain of the headline workload, 256 states: two sampled states against the oracle (FP32),
    and the Christoffel identity and dM/dq = the (q, qdd) block at every state (FP64)."""
    n, B = 32, 256
    print(f"case: hessian {n} links x {B} states", flush=True)
    ch = synth.make_chains([n], 7)
    chr_ = synth.Chains(*(a.astype(np.float32).astype(np.float64) for a in (ch.placement, ch.twist, ch.inertia)),
                        ch.link_ptr)
    st = synth.make_states((B, n), 7).rounded()
    m32 = api.Model(ch, device, torch.float32)
    q, qd, qdd = (dev(a, device, torch.float32) for a in (st.q, st.qd, st.qdd))
    H = api.rnea_id_hessian(m32, q, qd, qdd)
    assert api.read_status(device) == 0
    for s in (0, B - 1):
        ref = oracle_blocks(chr_, st.q[s], st.qd[s], st.qdd[s])
        assert worst({b: H[b][s].cpu().numpy().astype(np.float64) for b in BLOCKS}, ref) <= 5e-5, s

    m64 = api.Model(chr_, device, torch.float64)
    q, qd, qdd = (dev(a, device, torch.float64) for a in (st.q, st.qd, st.qdd))
    H = api.rnea_id_hessian(m64, q, qd, qdd, blocks=("qd_qd", "q_qdd"), base_vel=np.zeros(6))
    Hvv, Hqa = H["qd_qd"].cpu().numpy(), H["q_qdd"].cpu().numpy()
    assert christoffel_residual(Hvv, Hqa) <= 1e-10
    h = 1e-6
    for j in (0, 13, n - 1):
        e = torch.zeros(n, dtype=torch.float64, device=device)
        e[j] = h
        dM = ((api.mass_matrix(m64, q + e) - api.mass_matrix(m64, q - e)) / (2 * h)).cpu().numpy()  # [s, i, k]
        assert np.abs(dM - Hqa[:, :, j, :]).max() <= 1e-7 * np.abs(Hqa).max(), j
