"""Seeded synthetic serial chains and states.

The paper initialises "robot configuration parameters such as twists" at
random (Sec. V) and times many randomised joint inputs; it names no dataset.
This module is the one input generator that both the GPU path and the FP64
oracle are fed from. It holds no dynamics arithmetic: it only draws numbers.

Per link, in draw order (one ``numpy.random.Generator`` per chain, keyed by
``(seed, 0, chain)``):

1. joint axis direction w = normalize(N(0, I3));
2. a point r ~ U[-0.3, 0.3]^3 on the axis; twist S = (r x w, w) (revolute,
   zero pitch, twist order (v, w) as in Sec. III-C);
3. placement M_i: rotation = normalize(N(0, I4)) quaternion with w >= 0,
   translation ~ U[-0.5, 0.5]^3;
4. mass m ~ U[0.5, 5] kg, centre of mass c ~ U[-0.1, 0.1]^3 m (frame i);
5. principal moments ~ U[0.01, 0.1]^3 kg m^2, all three re-drawn together
   until each is <= the sum of the other two;
6. principal-axis rotation Q = normalize(N(0, I4)); I_c = Q diag Q^T, stored
   as (xx, yy, zz, xy, xz, yz).

States (stream 1): q ~ U[-pi, pi], qd ~ N(0, 1), qdd ~ N(0, 1),
tau ~ N(0, 10^2). Rollout torques (stream 2 + t): tau_t ~ N(0, 10^2).

Arrays come in FP64 and rounded to FP32; the oracle consumes the rounded
values promoted to FP64 so that a GPU-vs-oracle difference measures kernel
arithmetic only.
"""

from __future__ import annotations

import dataclasses

import numpy as np

BASE_SEED = 160904493
GRAVITY = 9.81


def _rng(seed: int, stream: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(entropy=seed, spawn_key=(stream, sub))))


def _quat_to_matrix(qw, qx, qy, qz):
    return np.array([
        [1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)],
        [2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)],
        [2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)],
    ])


def _unit_quat(rng):
    qv = rng.standard_normal(4)
    qv /= np.linalg.norm(qv)
    if qv[0] < 0:
        qv = -qv
    return qv


@dataclasses.dataclass
class Chains:
    """A set of serial chains in CSR form over links.

    placement: [L, 7]  (quaternion w, x, y, z of M_i's rotation; translation)
    twist:     [L, 6]  S_i = (v, w) in frame i
    inertia:   [L, 10] (m, c_x, c_y, c_z, I_xx, I_yy, I_zz, I_xy, I_xz, I_yz),
               I about the centre of mass in frame-i axes
    link_ptr:  [n_chains + 1] int32 offsets; chain c owns links
               link_ptr[c] .. link_ptr[c+1]-1, base to tip.
    """

    placement: np.ndarray
    twist: np.ndarray
    inertia: np.ndarray
    link_ptr: np.ndarray

    @property
    def n_chains(self) -> int:
        return len(self.link_ptr) - 1

    @property
    def n_links_total(self) -> int:
        return int(self.link_ptr[-1])

    def lengths(self) -> np.ndarray:
        return np.diff(self.link_ptr)

    def astype(self, dtype) -> "Chains":
        return Chains(self.placement.astype(dtype), self.twist.astype(dtype),
                      self.inertia.astype(dtype), self.link_ptr.copy())

    def rounded(self) -> "Chains":
        """FP32-rounded values, promoted back to FP64."""
        return self.astype(np.float32).astype(np.float64)

    def chain(self, c: int) -> "Chains":
        a, b = int(self.link_ptr[c]), int(self.link_ptr[c + 1])
        return Chains(self.placement[a:b], self.twist[a:b], self.inertia[a:b],
                      np.array([0, b - a], dtype=np.int32))


def _draw_link(rng):
    w = rng.standard_normal(3)
    w /= np.linalg.norm(w)
    r = rng.uniform(-0.3, 0.3, 3)
    twist = np.concatenate([np.cross(r, w), w])
    quat = _unit_quat(rng)
    trans = rng.uniform(-0.5, 0.5, 3)
    m = rng.uniform(0.5, 5.0)
    c = rng.uniform(-0.1, 0.1, 3)
    while True:
        d = rng.uniform(0.01, 0.1, 3)
        if d[0] <= d[1] + d[2] and d[1] <= d[0] + d[2] and d[2] <= d[0] + d[1]:
            break
    Q = _quat_to_matrix(*_unit_quat(rng))
    Ic = Q @ np.diag(d) @ Q.T
    inertia = np.array([m, c[0], c[1], c[2], Ic[0, 0], Ic[1, 1], Ic[2, 2], Ic[0, 1], Ic[0, 2], Ic[1, 2]])
    return np.concatenate([quat, trans]), twist, inertia


def make_chains(lengths, seed: int = BASE_SEED) -> Chains:
    """One chain per entry of ``lengths``; chain c draws from stream (seed, 0, c)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    link_ptr = np.zeros(len(lengths) + 1, dtype=np.int32)
    link_ptr[1:] = np.cumsum(lengths)
    L = int(link_ptr[-1])
    pl = np.empty((L, 7))
    tw = np.empty((L, 6))
    ine = np.empty((L, 10))
    for c, n in enumerate(lengths):
        rng = _rng(seed, 0, c)
        for k in range(int(n)):
            i = link_ptr[c] + k
            pl[i], tw[i], ine[i] = _draw_link(rng)
    return Chains(pl, tw, ine, link_ptr)


@dataclasses.dataclass
class States:
    """Joint-space states; arrays are [n_states, n] (uniform) or [L] (ragged)."""

    q: np.ndarray
    qd: np.ndarray
    qdd: np.ndarray
    tau: np.ndarray

    def astype(self, dtype) -> "States":
        return States(*(a.astype(dtype) for a in (self.q, self.qd, self.qdd, self.tau)))

    def rounded(self) -> "States":
        return self.astype(np.float32).astype(np.float64)


def make_states(shape, seed: int = BASE_SEED) -> States:
    rng = _rng(seed, 1)
    q = rng.uniform(-np.pi, np.pi, shape)
    qd = rng.standard_normal(shape)
    qdd = rng.standard_normal(shape)
    tau = 10.0 * rng.standard_normal(shape)
    return States(q, qd, qdd, tau)


def rollout_torques(t: int, shape, seed: int = BASE_SEED, dtype=np.float32) -> np.ndarray:
    """Torque input of rollout step t, N(0, 10^2), stream (seed, 2 + t)."""
    return (10.0 * _rng(seed, 2 + t).standard_normal(shape, dtype=np.float64)).astype(dtype)


def base_acceleration() -> np.ndarray:
    """Gravity -9.81 z entered as the base acceleration dV_0 = (0, 0, +9.81, 0, 0, 0)."""
    return np.array([0.0, 0.0, GRAVITY, 0.0, 0.0, 0.0])


# ---- the workloads -----------------------------------------------------------

def config_seed(k: int) -> int:
    return BASE_SEED + k


def workload_fp64_7link(batch: int = 64):
    """7-link chain, 64 states (FP64 correctness anchor)."""
    s = config_seed(1)
    return make_chains([7], s), make_states((batch, 7), s)


def workload_32link(batch: int = 16384):
    """32-link chain shared by 16384 states (ID + FD)."""
    s = config_seed(2)
    return make_chains([32], s), make_states((batch, 32), s)


def workload_uneven(n_chains: int = 4096, lo: int = 10, hi: int = 100):
    """n_chains chains with link counts uniform in [lo, hi], one state each."""
    s = config_seed(3)
    lengths = _rng(s, 9).integers(lo, hi + 1, n_chains)
    ch = make_chains(lengths, s)
    return ch, make_states((ch.n_links_total,), s)


def workload_50link(batch: int = 8192):
    """50-link chain, 8192 states (FD + adjoint)."""
    s = config_seed(4)
    return make_chains([50], s), make_states((batch, 50), s)


def workload_100link_rollout(batch: int = 65536):
    """100-link chain, 65536 states; torques per step from rollout_torques."""
    s = config_seed(5)
    return make_chains([100], s), make_states((batch, 100), s)
