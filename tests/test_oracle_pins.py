"""Pins of the FP64 oracle against facts fixed outside it (CPU only).

Each test would fail for a plausible slip in the oracle: a wrong sign or
transpose in Ad / ad, a wrong parallel-axis term in J, gravity entering with
the wrong sign or frame, a dropped velocity-product term, a wrong index in the
articulated-body recursions or in the Euler update.
"""

import dataclasses

import numpy as np
import pytest

import oracle
from paper_1609_04493_amd import synth
from tests import fk_textbook as fk


@dataclasses.dataclass
class Ch:
    placement: np.ndarray
    twist: np.ndarray
    inertia: np.ndarray
    link_ptr: np.ndarray


def small_chain(n, seed):
    return synth.make_chains([n], seed)


def rand_state(n, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-np.pi, np.pi, n), rng.standard_normal(n), rng.standard_normal(n)


NO_G = np.zeros(6)


# ---- one rigid link about a fixed axis: closed form ---------------------------------

@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_one_link_closed_form(seed):
    """A single body on a fixed revolute axis: tau = I_axis qdd - w.((c - r) x m g) (no velocity terms)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(3); w /= np.linalg.norm(w)
    r = rng.uniform(-0.3, 0.3, 3)
    quat = rng.standard_normal(4); quat /= np.linalg.norm(quat)
    trans = rng.uniform(-0.5, 0.5, 3)
    m = rng.uniform(0.5, 5); c = rng.uniform(-0.1, 0.1, 3)
    A = rng.standard_normal((3, 3)); Ic = A @ A.T * 0.05 + 0.01 * np.eye(3)
    ch = Ch(np.concatenate([quat, trans])[None], np.concatenate([np.cross(r, w), w])[None],
            np.array([[m, *c, Ic[0, 0], Ic[1, 1], Ic[2, 2], Ic[0, 1], Ic[0, 2], Ic[1, 2]]]), np.array([0, 1], np.int32))
    q, qd, qdd = rng.uniform(-np.pi, np.pi), rng.standard_normal(), rng.standard_normal()
    tau = oracle.rnea1(ch, [q], [qd], [qdd])[0]

    # independent closed form in base coordinates
    T = fk.link_frames(ch, np.array([q]))[0]
    R01, p01 = T[:3, :3], T[:3, 3]
    RM = fk.placement_matrix(ch.placement[0])[:3, :3]
    w_w = RM @ w
    r_w = RM @ r + trans
    c_w = R01 @ c + p01
    I_axis = w @ Ic @ w + m * np.sum(np.cross(w, c - r) ** 2)
    g_w = np.array([0, 0, -9.81])
    expect = I_axis * qdd - w_w @ np.cross(c_w - r_w, m * g_w)
    assert abs(tau - expect) <= 1e-13 * max(1.0, abs(expect))
    # and no dependence on the joint rate
    tau2 = oracle.rnea1(ch, [q], [5.0 * qd + 1.0], [qdd])[0]
    assert abs(tau2 - tau) <= 1e-13 * max(1.0, abs(expect))


# ---- Euler-Lagrange equations of the textbook energies --------------------------------

@pytest.mark.parametrize("n,seed", [(2, 11), (4, 12), (6, 13)])
def test_rnea_equals_euler_lagrange(n, seed):
    """tau_RNEA(q, qd, qdd) = d/dt dL/dqd - dL/dq with L from expm forward kinematics (gravity on)."""
    ch = small_chain(n, seed)
    q, qd, qdd = rand_state(n, seed)
    tau = oracle.rnea1(ch, q, qd, qdd)
    tau_L = fk.lagrange_torque(ch, q, qd, qdd)
    assert np.linalg.norm(tau - tau_L) <= 1e-7 * np.linalg.norm(tau_L)


@pytest.mark.parametrize("n,seed", [(3, 21), (7, 22)])
def test_mass_matrix_matches_textbook(n, seed):
    ch = small_chain(n, seed)
    q, _, _ = rand_state(n, seed)
    M = oracle.mass_matrix(ch, q)
    Mfk = fk.mass_matrix(ch, q)
    assert np.abs(M - Mfk).max() <= 1e-12 * np.abs(Mfk).max()
    assert np.abs(M - M.T).max() <= 1e-13 * np.abs(M).max()
    np.linalg.cholesky(M)  # positive definite


@pytest.mark.parametrize("n,seed", [(5, 31), (9, 32)])
def test_gravity_torque_is_potential_gradient(n, seed):
    """tau(q, 0, 0) = dU/dq with U = sum m g z(c_i) from the textbook forward kinematics."""
    ch = small_chain(n, seed)
    q, _, _ = rand_state(n, seed)
    tau = oracle.rnea1(ch, q, np.zeros(n), np.zeros(n))
    h = 1e-6
    dU = np.array([(fk.potential_energy(ch, q + h * e) - fk.potential_energy(ch, q - h * e)) / (2 * h) for e in np.eye(n)])
    assert np.linalg.norm(tau - dU) <= 1e-8 * np.linalg.norm(dU)


@pytest.mark.parametrize("n,seed", [(4, 41), (8, 42)])
def test_power_balance(n, seed):
    """Gravity off: qd^T tau = sum V_i^T J_i dV_i exactly, and = dE/dt (central difference of E)."""
    ch = small_chain(n, seed)
    q, qd, qdd = rand_state(n, seed)
    tr = oracle.rnea_trace(ch, q, qd, qdd, dV0=NO_G)
    tau = tr["tau"][1:]
    power = qd @ tau
    # sum V^T Fhat = sum V^T J dV (the gyroscopic term does no work); the identity is the telescoped recursion
    s = sum(tr["V"][i] @ tr["Fhat"][i] for i in range(1, n + 1))
    terms = sum(abs(tr["V"][i]) @ abs(tr["Fhat"][i]) for i in range(1, n + 1))
    assert abs(power - s) <= 1e-12 * terms
    h = 1e-5
    dEdt = (fk.kinetic_energy(ch, q + h * qd, qd + h * qdd) - fk.kinetic_energy(ch, q - h * qd, qd - h * qdd)) / (2 * h)
    assert abs(power - dEdt) <= 1e-7 * max(1.0, abs(power))


@pytest.mark.parametrize("n,seed", [(7, 51), (32, 52), (50, 53)])
def test_fd_inverts_id_and_equals_jsiia(n, seed):
    ch = small_chain(n, seed).rounded()
    q, qd, qdd = rand_state(n, seed)
    tau = oracle.rnea1(ch, q, qd, qdd)
    qdd_aba = oracle.aba1(ch, q, qd, tau)
    qdd_jsi = oracle.jsiia1(ch, q, qd, tau)
    assert np.linalg.norm(qdd_aba - qdd) <= 1e-9 * np.linalg.norm(qdd)
    assert np.linalg.norm(qdd_aba - qdd_jsi) <= 1e-9 * np.linalg.norm(qdd)


def test_fd_with_base_motion_and_tip_wrench():
    """FD(q, qd, ID(q, qd, qdd, V0, dV0, F_tip), V0, dV0, F_tip) = qdd with all boundary terms non-zero."""
    n = 6
    ch = small_chain(n, 61)
    q, qd, qdd = rand_state(n, 61)
    rng = np.random.default_rng(61)
    V0, dV0, Ft = rng.standard_normal(6), rng.standard_normal(6), rng.standard_normal(6)
    tau = oracle.rnea1(ch, q, qd, qdd, V0, dV0, Ft)
    assert np.linalg.norm(oracle.aba1(ch, q, qd, tau, V0, dV0, Ft) - qdd) <= 1e-10 * np.linalg.norm(qdd)
    assert np.linalg.norm(oracle.jsiia1(ch, q, qd, tau, V0, dV0, Ft) - qdd) <= 1e-10 * np.linalg.norm(qdd)


def test_tip_wrench_is_a_static_load():
    """A tip wrench F enters as J_tip^T F: tau(F) - tau(0) = Jb_n^T F with the body Jacobian of link n."""
    n = 5
    ch = small_chain(n, 71)
    q, qd, qdd = rand_state(n, 71)
    F = np.random.default_rng(71).standard_normal(6)
    d = oracle.rnea1(ch, q, qd, qdd, Ftip=F) - oracle.rnea1(ch, q, qd, qdd)
    Jb = fk.body_jacobians(ch, q)[-1]
    assert np.linalg.norm(d - Jb.T @ F) <= 1e-11 * np.linalg.norm(d)


def test_base_frame_invariance():
    """Re-expressing the base by T (M_1 -> T M_1, dV0 -> Ad_T dV0) leaves tau and qdd unchanged."""
    n = 6
    ch = small_chain(n, 81)
    q, qd, qdd = rand_state(n, 81)
    rng = np.random.default_rng(81)
    qt = rng.standard_normal(4); qt /= np.linalg.norm(qt)
    T = fk.placement_matrix(np.concatenate([qt, rng.uniform(-1, 1, 3)]))
    M1 = fk.placement_matrix(ch.placement[0])
    TM = T @ M1
    from scipy.spatial.transform import Rotation
    x, y, z, w = Rotation.from_matrix(TM[:3, :3]).as_quat()
    pl = ch.placement.copy()
    pl[0] = [w, x, y, z, *TM[:3, 3]]
    ch2 = Ch(pl, ch.twist, ch.inertia, ch.link_ptr)
    R, p = T[:3, :3], T[:3, 3]
    AdT = np.zeros((6, 6)); AdT[:3, :3] = R; AdT[3:, 3:] = R
    AdT[:3, 3:] = np.array([[0, -p[2], p[1]], [p[2], 0, -p[0]], [-p[1], p[0], 0]]) @ R
    dV0 = AdT @ oracle.GRAVITY_ACC
    tau = oracle.rnea1(ch, q, qd, qdd)
    tau2 = oracle.rnea1(ch2, q, qd, qdd, dV0=dV0)
    assert np.linalg.norm(tau - tau2) <= 1e-12 * np.linalg.norm(tau)
    assert np.linalg.norm(oracle.aba1(ch2, q, qd, tau, dV0=dV0) - qdd) <= 1e-10 * np.linalg.norm(qdd)


def test_id_affine_in_qdd_with_slope_M():
    n = 8
    ch = small_chain(n, 91)
    q, qd, qdd = rand_state(n, 91)
    M = oracle.mass_matrix(ch, q)
    t0 = oracle.rnea1(ch, q, qd, np.zeros(n))
    assert np.linalg.norm(oracle.rnea1(ch, q, qd, qdd) - (t0 + M @ qdd)) <= 1e-12 * np.linalg.norm(t0 + M @ qdd)


def test_id_homogeneous_in_mass_and_inertia():
    """Scaling every m and I_c by a (centres of mass fixed) scales tau by a."""
    n = 6
    ch = small_chain(n, 92)
    q, qd, qdd = rand_state(n, 92)
    a = 2.75
    ine = ch.inertia.copy(); ine[:, 0] *= a; ine[:, 4:] *= a
    ch2 = Ch(ch.placement, ch.twist, ine, ch.link_ptr)
    t1, t2 = oracle.rnea1(ch, q, qd, qdd), oracle.rnea1(ch2, q, qd, qdd)
    assert np.linalg.norm(t2 - a * t1) <= 1e-13 * np.linalg.norm(a * t1)


def test_kinetic_energy_quadratic_form():
    n = 7
    ch = small_chain(n, 93)
    q, qd, _ = rand_state(n, 93)
    M = oracle.mass_matrix(ch, q)
    E = fk.kinetic_energy(ch, q, qd)
    assert abs(0.5 * qd @ M @ qd - E) <= 1e-12 * E


# ---- rollout: constant-acceleration closed form ---------------------------------------

def test_rollout_semi_implicit_euler_closed_form():
    """One link, no gravity, constant torque: qdd = tau/I is constant and semi-implicit Euler gives
    qd_T = qd0 + T dt a,  q_T = q0 + T dt qd0 + dt^2 a T (T + 1) / 2 (explicit Euler would give T (T - 1) / 2)."""
    ch = small_chain(1, 101)
    I_axis = oracle.mass_matrix(ch, [0.3])[0, 0]
    steps, dt, tau = 37, 1e-2, 2.5
    qT, qdT = oracle.rollout1(ch, steps, dt, np.array([0.3]), np.array([-0.7]), np.full((steps, 1), tau), dV0=NO_G)
    a = tau / I_axis
    assert abs(qdT[0] - (-0.7 + steps * dt * a)) <= 1e-12
    assert abs(qT[0] - (0.3 + steps * dt * -0.7 + dt * dt * a * steps * (steps + 1) / 2)) <= 1e-12


def test_batched_entry_points_match_single():
    ch, st = synth.workload_fp64_7link(8)
    tau = oracle.rnea(ch, st.q, st.qd, st.qdd, threads=3)
    qdd = oracle.aba(ch, st.q, st.qd, st.tau)
    for s in range(8):
        assert np.array_equal(tau[s], oracle.rnea1(ch, st.q[s], st.qd[s], st.qdd[s]))
        assert np.array_equal(qdd[s], oracle.aba1(ch, st.q[s], st.qd[s], st.tau[s]))


def test_ragged_batch_matches_per_chain():
    chs = synth.make_chains([3, 7, 1, 5], seed=5)
    st = synth.make_states((chs.n_links_total,), seed=5)
    tau = oracle.rnea(chs, st.q, st.qd, st.qdd)
    for c in range(4):
        a, b = chs.link_ptr[c], chs.link_ptr[c + 1]
        assert np.array_equal(tau[a:b], oracle.rnea1(chs.chain(c), st.q[a:b], st.qd[a:b], st.qdd[a:b]))
