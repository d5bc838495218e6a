"""GPU parity of the adjoint kernels against the oracle's complex-step derivatives (needs an MI355X).

FP64 kernels must match to rounding. FP32 tolerances are per output, relative
per state (||x - x*|| / ||x*||). For the forward-dynamics adjoint, q_bar is a
strongly cancelling sum -(dtau/dq)^T M^-1 qdd_bar whose FP32 error grows with
cond(M) (~1e4-1e5 here): it is held to 1e-3, the other outputs to 1e-4.

Full-size launches use a cotangent that is zero except on sampled states, so
the batch-summed inertia gradient equals the oracle's sum over those states.
"""

import os

import numpy as np
import pytest
import torch

import oracle
from oracle import grad
from paper_1609_04493_amd import api, autograd, synth

pytestmark = pytest.mark.gpu
THREADS = min(16, len(os.sched_getaffinity(0)))


def dev_t(a, device, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(device)


def rel(x, ref, floor=0.0):
    """Relative error ||x - ref|| / ||ref||. `floor` is an absolute scale passed only for an output that
    vanishes analytically, whose reference is rounding noise: a one-link chain's qd_bar. For one link,
    d tau/d qd = -S^T J ad_S X V0 (through dV) + (ad_S X V0)^T J S (through the gyroscopic term) = 0, for any
    base motion, so the adjoint's qd_bar is zero too."""
    num = np.linalg.norm(np.asarray(x, np.float64) - ref)
    den = max(np.linalg.norm(ref), floor)
    return num / den if den > 0 else num


def vanishing_floor(k, n_links):
    """The floor of output k (0 q_bar, 1 qd_bar, ...) of an n-link chain."""
    return 1e-3 if (k == 1 and n_links == 1) else 0.0


def id_refs(ch, st, bar, idx):
    out = [np.zeros((len(idx), st.q.shape[1])) for _ in range(3)]
    pib = np.zeros((st.q.shape[1], 10))
    for k, s in enumerate(idx):
        r = grad.rnea_vjp(ch, st.q[s], st.qd[s], st.qdd[s], bar[s])
        for j in range(3):
            out[j][k] = r[j]
        pib += r[3]
    return out, pib


def fd_refs(ch, st, bar, idx):
    out = [np.zeros((len(idx), st.q.shape[1])) for _ in range(3)]
    pib = np.zeros((st.q.shape[1], 10))
    for k, s in enumerate(idx):
        r = grad.aba_vjp(ch, st.q[s], st.qd[s], st.tau[s], bar[s])
        for j in range(3):
            out[j][k] = r[j]
        pib += r[3]
    return out, pib


@pytest.mark.parametrize("B", [64, 67])
def test_fp64_id_and_fd_vjp_7_links(device, B):
    print(f"case: fp64 vjp 7 links B={B}", flush=True)
    ch, st = synth.workload_fp64_7link(B)
    bar = np.random.default_rng(B).standard_normal((B, 7))
    model = api.Model(ch, device, torch.float64)
    d = lambda a: dev_t(a, device, torch.float64)
    qb, qdb, qddb, pib = (x.cpu().numpy() for x in api.rnea_id_vjp(model, d(st.q), d(st.qd), d(st.qdd), d(bar)))
    idx = np.arange(B)
    (rq, rqd, rqdd), rpi = id_refs(ch, st, bar, idx)
    for x, r in ((qb, rq), (qdb, rqd), (qddb, rqdd)):
        assert max(rel(x[s], r[s]) for s in idx) <= 1e-11
    assert rel(pib, rpi) <= 1e-11
    qdd = oracle.aba(ch, st.q, st.qd, st.tau)
    qb, qdb, tb, pib = (x.cpu().numpy() for x in api.aba_fd_vjp(model, d(st.q), d(st.qd), d(qdd), d(bar)))
    (rq, rqd, rt), rpi = fd_refs(ch, st, bar, idx)
    for x, r in ((qb, rq), (qdb, rqd), (tb, rt)):
        assert max(rel(x[s], r[s]) for s in idx) <= 1e-10
    assert rel(pib, rpi) <= 1e-10


def test_fp32_id_vjp_32_links_full_batch_sparse_cotangent(device):
    print("case: fp32 id vjp 32 links x 16384", flush=True)
    ch, st = synth.workload_32link(16384)
    idx = np.random.default_rng(5).choice(16384, 24, replace=False)
    bar = np.zeros((16384, 32))
    bar[idx] = np.random.default_rng(6).standard_normal((24, 32))
    model = api.Model(ch, device, torch.float32)
    d = lambda a: dev_t(a, device, torch.float32)
    qb, qdb, qddb, pib = (x.cpu().numpy() for x in api.rnea_id_vjp(model, d(st.q), d(st.qd), d(st.qdd), d(bar)))
    cr, sr = ch.rounded(), st.rounded()
    (rq, rqd, rqdd), rpi = id_refs(cr, sr, bar, idx)
    errs = {k: max(rel(x[s], r[k2]) for k2, s in enumerate(idx)) for k, x, r in
            (("q", qb, rq), ("qd", qdb, rqd), ("qdd", qddb, rqdd))}
    errs["pi"] = rel(pib, rpi)
    print("fp32 ID vjp errors", errs, flush=True)
    assert max(errs.values()) <= 1e-4
    zero = np.setdiff1d(np.arange(16384), idx)
    assert np.abs(qb[zero]).max() == 0 and np.abs(qddb[zero]).max() == 0


def test_fp32_fd_vjp_50_links_8192_states(device):
    """The 50-link, 8192-state workload: FD + adjoint of L = ||qdd||^2 (cotangent 2 qdd) on sampled states."""
    print("case: fp32 fd vjp 50 links x 8192", flush=True)
    ch, st = synth.workload_50link(8192)
    model = api.Model(ch, device, torch.float32)
    d = lambda a: dev_t(a, device, torch.float32)
    q, qd, tau = d(st.q), d(st.qd), d(st.tau)
    qdd = api.aba_fd(model, q, qd, tau)
    idx = np.random.default_rng(7).choice(8192, 12, replace=False)
    mask = torch.zeros(8192, 1, device=device)
    mask[torch.as_tensor(idx)] = 1.0
    bar = (2.0 * qdd * mask).contiguous()
    qb, qdb, tb, pib = (x.cpu().numpy() for x in api.aba_fd_vjp(model, q, qd, qdd, bar))
    cr, sr = ch.rounded(), st.rounded()
    bar_np = bar.cpu().numpy().astype(np.float64)
    (rq, rqd, rt), rpi = fd_refs(cr, sr, bar_np, idx)
    errs = {k: max(rel(x[s], r[k2]) for k2, s in enumerate(idx)) for k, x, r in
            (("q", qb, rq), ("qd", qdb, rqd), ("tau", tb, rt))}
    errs["pi"] = rel(pib, rpi)
    print("fp32 FD vjp errors (50 links)", errs, flush=True)
    assert errs["q"] <= 1e-3
    assert max(errs["qd"], errs["tau"], errs["pi"]) <= 1e-4


def test_fp64_fd_vjp_vs_central_differences(device):
    """d/de L(q + e dq, qd + e dqd, tau + e dtau), L = ||FD||^2, by FP64 central differences (h = 1e-6) on the GPU."""
    print("case: fp64 fd vjp vs central differences", flush=True)
    ch = synth.make_chains([50], 11)
    st = synth.make_states((8, 50), 11)
    model = api.Model(ch, device, torch.float64)
    d = lambda a: dev_t(a, device, torch.float64)
    q, qd, tau = d(st.q), d(st.qd), d(st.tau)
    qdd = api.aba_fd(model, q, qd, tau)
    qb, qdb, tb, _ = api.aba_fd_vjp(model, q, qd, qdd, (2 * qdd).contiguous(), want_inertia=False)
    rng = np.random.default_rng(12)
    dq, dqd, dtau = (d(rng.standard_normal((8, 50))) for _ in range(3))
    h = 1e-6
    Lp = (api.aba_fd(model, q + h * dq, qd + h * dqd, tau + h * dtau) ** 2).sum(1)
    Lm = (api.aba_fd(model, q - h * dq, qd - h * dqd, tau - h * dtau) ** 2).sum(1)
    cd = ((Lp - Lm) / (2 * h)).cpu().numpy()
    adj = ((qb * dq).sum(1) + (qdb * dqd).sum(1) + (tb * dtau).sum(1)).cpu().numpy()
    assert np.abs(cd - adj).max() <= 1e-5 * np.abs(adj).max()


def test_ragged_chains_vjp_direct_inertia_rows(device):
    print("case: ragged vjp", flush=True)
    ch = synth.make_chains([3, 10, 1, 17, 7], 21)
    st = synth.make_states((ch.n_links_total,), 21)
    bar = np.random.default_rng(21).standard_normal(ch.n_links_total)
    model = api.Model(ch, device, torch.float64)
    d = lambda a: dev_t(a, device, torch.float64)
    qb, qdb, qddb, pib = (x.cpu().numpy() for x in api.rnea_id_vjp(model, d(st.q), d(st.qd), d(st.qdd), d(bar)))
    qdd = oracle.aba(ch, st.q, st.qd, st.tau)
    fb, fdb, ftb, fpib = (x.cpu().numpy() for x in api.aba_fd_vjp(model, d(st.q), d(st.qd), d(qdd), d(bar)))
    for c in range(ch.n_chains):
        a, b = ch.link_ptr[c], ch.link_ptr[c + 1]
        sub = ch.chain(c)
        r = grad.rnea_vjp(sub, st.q[a:b], st.qd[a:b], st.qdd[a:b], bar[a:b])
        for k, (x, y) in enumerate(zip((qb[a:b], qdb[a:b], qddb[a:b], pib[a:b]), r)):
            assert rel(x, y, vanishing_floor(k, b - a)) <= 1e-11
        r = grad.aba_vjp(sub, st.q[a:b], st.qd[a:b], st.tau[a:b], bar[a:b])
        for k, (x, y) in enumerate(zip((fb[a:b], fdb[a:b], ftb[a:b], fpib[a:b]), r)):
            assert rel(x, y, vanishing_floor(k, b - a)) <= 1e-10


def test_autograd_functions_match_vjp_kernels(device):
    print("case: autograd", flush=True)
    ch, st = synth.workload_fp64_7link(32)
    model = api.Model(ch, device, torch.float64)
    d = lambda a: dev_t(a, device, torch.float64).requires_grad_(True)
    q, qd, tau, ine = d(st.q), d(st.qd), d(st.tau), d(ch.inertia)
    qdd = autograd.forward_dynamics(model, q, qd, tau, ine)
    loss = (qdd ** 2).sum()
    gq, gqd, gt, gpi = torch.autograd.grad(loss, (q, qd, tau, ine))
    for s in range(0, 32, 8):
        r = grad.aba_vjp(ch, st.q[s], st.qd[s], st.tau[s], 2 * qdd[s].detach().cpu().numpy())
        for x, y in zip((gq[s], gqd[s], gt[s]), r[:3]):
            assert rel(x.cpu().numpy(), y) <= 1e-10
    tauo = autograd.inverse_dynamics(model, q, qd, qdd.detach(), ine)
    g2 = torch.autograd.grad(tauo.sum(), (q, ine))
    r = grad.rnea_vjp(ch, st.q[3], st.qd[3], qdd[3].detach().cpu().numpy(), np.ones(7))
    assert rel(g2[0][3].cpu().numpy(), r[0]) <= 1e-10


def test_inertia_gradient_is_deterministic(device):
    ch, st = synth.workload_32link(4096)
    model = api.Model(ch, device, torch.float32)
    d = lambda a: dev_t(a, device, torch.float32)
    bar = d(np.random.default_rng(3).standard_normal((4096, 32)))
    a = api.rnea_id_vjp(model, d(st.q), d(st.qd), d(st.qdd), bar)[3].cpu().numpy()
    b = api.rnea_id_vjp(model, d(st.q), d(st.qd), d(st.qdd), bar)[3].cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("variant", [1, 2, 3])
def test_adjoint_variants(device, variant):
    """Every adjoint variant (one wavefront per 64 states; role split; plain, one launch per pass) against the
    oracle: FP64 with base motion
    and tip wrenches on ragged chains, and the FP32 32-link FD adjoint on sampled states of a full batch."""
    print(f"case: adjoint variant {variant}", flush=True)
    for op in (api.OP_RNEA_ID_VJP, api.OP_ABA_FD_VJP):
        api.set_launch(op, 0, 0, variant)
    try:
        ch = synth.make_chains([5, 12, 1, 30, 9], 33)
        st = synth.make_states((ch.n_links_total,), 33)
        rng = np.random.default_rng(33)
        bar = rng.standard_normal(ch.n_links_total)
        tip = rng.standard_normal((ch.n_chains, 6))
        V0, dV0 = rng.standard_normal(6), rng.standard_normal(6)
        model = api.Model(ch, device, torch.float64)
        d = lambda a: dev_t(a, device, torch.float64)
        kw = dict(base_vel=tuple(V0), base_acc=tuple(dV0), tip=d(tip))
        qb, qdb, qddb, pib = (x.cpu().numpy() for x in
                              api.rnea_id_vjp(model, d(st.q), d(st.qd), d(st.qdd), d(bar), **kw))
        qdd = np.zeros_like(st.q)
        for c in range(ch.n_chains):
            a, b = ch.link_ptr[c], ch.link_ptr[c + 1]
            qdd[a:b] = oracle.aba1(ch.chain(c), st.q[a:b], st.qd[a:b], st.tau[a:b], V0, dV0, tip[c])
        fb, fdb, ftb, fpib = (x.cpu().numpy() for x in
                              api.aba_fd_vjp(model, d(st.q), d(st.qd), d(qdd), d(bar), **kw))
        for c in range(ch.n_chains):
            a, b = ch.link_ptr[c], ch.link_ptr[c + 1]
            sub = ch.chain(c)
            r = grad.rnea_vjp(sub, st.q[a:b], st.qd[a:b], st.qdd[a:b], bar[a:b], V0, dV0, tip[c])
            for k, (x, y) in enumerate(zip((qb[a:b], qdb[a:b], qddb[a:b], pib[a:b]), r)):
                assert rel(x, y, vanishing_floor(k, b - a)) <= 1e-11
            r = grad.aba_vjp(sub, st.q[a:b], st.qd[a:b], st.tau[a:b], bar[a:b], V0, dV0, tip[c])
            for k, (x, y) in enumerate(zip((fb[a:b], fdb[a:b], ftb[a:b], fpib[a:b]), r)):
                assert rel(x, y, vanishing_floor(k, b - a)) <= 1e-10
        ch, st = synth.workload_32link(16384)
        model = api.Model(ch, device, torch.float32)
        d = lambda a: dev_t(a, device, torch.float32)
        q, qd, tau = d(st.q), d(st.qd), d(st.tau)
        qdd = api.aba_fd(model, q, qd, tau)
        idx = np.random.default_rng(8).choice(16384, 12, replace=False)
        mask = torch.zeros(16384, 1, device=device)
        mask[torch.as_tensor(idx)] = 1.0
        barf = (2.0 * qdd * mask).contiguous()
        qb, qdb, tb, pib = (x.cpu().numpy() for x in api.aba_fd_vjp(model, q, qd, qdd, barf))
        cr, sr = ch.rounded(), st.rounded()
        (rq, rqd, rt), rpi = fd_refs(cr, sr, barf.cpu().numpy().astype(np.float64), idx)
        errs = {k: max(rel(x[s], r[k2]) for k2, s in enumerate(idx)) for k, x, r in
                (("q", qb, rq), ("qd", qdb, rqd), ("tau", tb, rt))}
        errs["pi"] = rel(pib, rpi)
        print(f"variant {variant}: fp32 FD adjoint errors (32 links)", errs, flush=True)
        assert errs["q"] <= 1e-3 and max(errs["qd"], errs["tau"], errs["pi"]) <= 1e-4
    finally:
        for op in (api.OP_RNEA_ID_VJP, api.OP_ABA_FD_VJP):
            api.set_launch(op, 0, 0, 0)


@pytest.mark.parametrize("n", [6, 60])
def test_adjoint_lds_levels(device, n):
    """The role-split adjoints at the LDS levels the chain length selects (FP64: 6 links, the adjoint sweep on
    two wavefronts with every hand-off in LDS; 60 links, no LDS hand-off), 67 states (a ragged second group),
    cotangents on 4 sampled states, against the oracle."""
    print(f"case: adjoint LDS level, fp64 {n} links", flush=True)
    ch = synth.make_chains([n], 60 + n)
    st = synth.make_states((67, n), 60 + n)
    model = api.Model(ch, device, torch.float64)
    d = lambda a: dev_t(a, device, torch.float64)
    idx = np.array([0, 17, 63, 66])
    bar = np.zeros((67, n))
    bar[idx] = np.random.default_rng(n).standard_normal((len(idx), n))
    qb, qdb, qddb, pib = (x.cpu().numpy() for x in api.rnea_id_vjp(model, d(st.q), d(st.qd), d(st.qdd), d(bar)))
    (rq, rqd, rqdd), rpi = id_refs(ch, st, bar, idx)
    for k, s in enumerate(idx):
        assert max(rel(qb[s], rq[k]), rel(qdb[s], rqd[k]), rel(qddb[s], rqdd[k])) <= 1e-10, s
    assert rel(pib, rpi) <= 1e-10
    qdd = oracle.aba(ch, st.q, st.qd, st.tau)
    fb, fdb, ftb, fpib = (x.cpu().numpy() for x in api.aba_fd_vjp(model, d(st.q), d(st.qd), d(qdd), d(bar)))
    (rq, rqd, rt), rpi = fd_refs(ch, st, bar, idx)
    for k, s in enumerate(idx):
        assert max(rel(fb[s], rq[k]), rel(fdb[s], rqd[k]), rel(ftb[s], rt[k])) <= 1e-10, s
    assert rel(fpib, rpi) <= 1e-10


def test_jacobian_mode_50_links_8192_states(device):
    """Full FD Jacobians of the 50-link, 8192-state workload by stacked one-hot cotangents: 64 sampled
    states against the oracle's complex-step Jacobians; at every state dqdd/dtau (= M^-1) times the ID
    Jacobian dtau/dqdd (= M) is the identity."""
    print("case: jacobian mode 50 links x 8192", flush=True)
    from paper_1609_04493_amd import jacobian
    ch, st = synth.workload_50link(8192)
    model = api.Model(ch, device, torch.float32)
    d = lambda a: dev_t(a, device, torch.float32)
    q, qd, tau = d(st.q), d(st.qd), d(st.tau)
    Jq, Jqd, Jt = jacobian.fd_jacobians(model, q, qd, tau)
    assert Jq.shape == (8192, 50, 50)
    cr, sr = ch.rounded(), st.rounded()
    idx = np.random.default_rng(9).choice(8192, 64, replace=False)
    f = lambda c, a, b, t: oracle.aba1(c, a, b, t)
    worst = {"q": 0.0, "qd": 0.0, "tau": 0.0}
    for s in idx:
        args = (sr.q[s], sr.qd[s], sr.tau[s])
        for k, (name, J) in enumerate((("q", Jq), ("qd", Jqd), ("tau", Jt))):
            ref = grad._jac(f, args, k, cr)
            worst[name] = max(worst[name], rel(J[s].cpu().numpy(), ref))
    print("jacobian mode rel errors (Frobenius, 64 states)", worst, flush=True)
    assert worst["q"] <= 1e-3 and worst["qd"] <= 1e-4 and worst["tau"] <= 1e-4
    qdd = api.aba_fd(model, q, qd, tau)
    _, _, M = jacobian.id_jacobians(model, q[:256], qd[:256], qdd[:256])
    eye = torch.eye(50, device=device).expand(256, 50, 50)
    prod = torch.bmm(M.contiguous(), Jt[:256].contiguous())
    err = ((prod - eye).norm(dim=(1, 2)) / 50 ** 0.5).max().item()
    print(f"FP32: max ||M M^-1 - I|| / sqrt(n) over 256 states: {err:.2e} (bounded by eps cond(M))", flush=True)
    assert err <= 1e-2
    # in FP64 the same identity holds to rounding, and M is symmetric
    m64 = api.Model(ch, device, torch.float64)
    d64 = lambda a: dev_t(a, device, torch.float64)
    q6, qd6, t6 = d64(st.q[:16]), d64(st.qd[:16]), d64(st.tau[:16])
    _, _, Minv = jacobian.fd_jacobians(m64, q6, qd6, t6)
    _, _, M6 = jacobian.id_jacobians(m64, q6, qd6, api.aba_fd(m64, q6, qd6, t6))
    eye6 = torch.eye(50, device=device, dtype=torch.float64).expand(16, 50, 50)
    assert (torch.bmm(M6.contiguous(), Minv.contiguous()) - eye6).abs().max().item() <= 1e-8
    assert (M6 - M6.transpose(1, 2)).abs().max().item() <= 1e-12 * M6.abs().max().item()
    assert (Minv - Minv.transpose(1, 2)).abs().max().item() <= 1e-9 * Minv.abs().max().item()


def test_autograd_sees_in_place_inertia_updates(device):
    """A learned inertia updated in place (as an optimizer step does) between two forwards: the second forward
    and its backward must use the new values, exactly as a freshly built model does; a backward still uses
    the tables of its own forward after another forward has re-prepared the model."""
    print("case: autograd in-place inertia update", flush=True)
    ch, st = synth.workload_fp64_7link(16)
    model = api.Model(ch, device, torch.float64)
    d = lambda a: dev_t(a, device, torch.float64)
    ine = d(ch.inertia).requires_grad_(True)
    q, qd, tau = d(st.q), d(st.qd), d(st.tau)
    qdd1 = autograd.forward_dynamics(model, q, qd, tau, ine)
    loss1 = (qdd1 ** 2).sum()
    with torch.no_grad():
        ine.mul_(1.5)  # same storage, new version
    qdd2 = autograd.forward_dynamics(model, q, qd, tau, ine)
    ch2 = synth.Chains(ch.placement, ch.twist, ch.inertia * 1.5, ch.link_ptr)
    fresh = api.Model(ch2, device, torch.float64)
    assert torch.equal(qdd2, api.aba_fd(fresh, q, qd, tau))
    assert not torch.allclose(qdd1, qdd2)
    # backward of the first forward: its own (unscaled) tables, against the oracle at the unscaled inertia
    g1 = torch.autograd.grad(loss1, (ine,))[0].cpu().numpy()
    ref = sum(grad.aba_vjp(ch, st.q[s], st.qd[s], st.tau[s], 2 * qdd1[s].detach().cpu().numpy())[3]
              for s in range(16))
    assert rel(g1, ref) <= 1e-10


def test_jacobian_entry_points_equal_one_hot_adjoints(device):
    """pdyn_rnea_id_jacobian / pdyn_aba_fd_jacobian: row i of each Jacobian equals the adjoint with cotangent
    e_i (FP64, base motion and tip wrenches, a batch that spans several expansion chunks), and the FD tau-block
    times the ID qdd-block is the identity (M^-1 M = I)."""
    print("case: jacobian entry points, fp64", flush=True)
    n, B = 9, 16000  # 2^17 / 9 = 14563 states per chunk: two chunks, the second ragged
    ch = synth.make_chains([n], 91)
    st = synth.make_states((B, n), 91)
    rng = np.random.default_rng(91)
    V0, dV0, tip = rng.standard_normal(6), rng.standard_normal(6), rng.standard_normal((B, 6))
    model = api.Model(ch, device, torch.float64)
    d = lambda a: dev_t(a, device, torch.float64)
    kw = dict(base_vel=tuple(V0), base_acc=tuple(dV0), tip=d(tip))
    q, qd, qdd, tau = d(st.q), d(st.qd), d(st.qdd), d(st.tau)
    Jq, Jqd, M = api.rnea_id_jacobian(model, q, qd, qdd, **kw)
    qddf = api.aba_fd(model, q, qd, tau, **kw)
    Fq, Fqd, Minv = api.aba_fd_jacobian(model, q, qd, qddf, **kw)
    for i in (0, 4, n - 1):
        e = torch.zeros((B, n), dtype=torch.float64, device=device)
        e[:, i] = 1.0
        qb, qdb, qddb, _ = api.rnea_id_vjp(model, q, qd, qdd, e, want_inertia=False, **kw)
        assert torch.equal(Jq[:, i, :], qb) and torch.equal(Jqd[:, i, :], qdb) and torch.equal(M[:, i, :], qddb)
        fb, fdb, tb, _ = api.aba_fd_vjp(model, q, qd, qddf, e, want_inertia=False, **kw)
        assert torch.equal(Fq[:, i, :], fb) and torch.equal(Fqd[:, i, :], fdb) and torch.equal(Minv[:, i, :], tb)
    eye = torch.eye(n, dtype=torch.float64, device=device).expand(B, n, n)
    assert (torch.bmm(Minv.contiguous(), M.contiguous()) - eye).abs().max().item() <= 1e-9
    s = 15000  # a state of the second chunk against the oracle's eq. (17) matrix
    ref = oracle.mass_matrix(ch, st.q[s])
    assert np.abs(M[s].cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
