"""The team kernels' segmented scans run on the CPU (host build of team.hpp) against the FP64 oracle.

The cross-lane scans are emulated with the kernels' own Kogge-Stone order and
combines, so these tests pin the arithmetic the GPU runs, for every segment
count from the serial fold (P = 1) to one link per lane.
"""

import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1609_04493_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kernel_cpu", "team_on_cpu.hip")


@pytest.fixture(scope="module")
def team_lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("tcpu") / "libteam_cpu.so")
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    extra = os.environ.get("PDYN_HOST_BUILD_FLAGS", "").split()  # set by the sanitizer run (test_sanitized_cpu)
    subprocess.run([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-host-only", *extra, "-o", out, SRC],
                   check=True)
    lib = ctypes.CDLL(out)
    for f in (lib.cpu_team_id_f32, lib.cpu_team_id_f64, lib.cpu_team_fd_f32, lib.cpu_team_fd_f64):
        f.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p] * 11
        f.restype = ctypes.c_int
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def team_id(lib, P, chains, st, dtype, tip=None, V0=None, dV0=None):
    dt = np.dtype(dtype)
    fn = lib.cpu_team_id_f64 if dt == np.float64 else lib.cpu_team_id_f32
    conv = lambda a: None if a is None else np.ascontiguousarray(a, dtype=dt)
    q = conv(st.q)
    n_states = q.shape[0] if chains.n_chains == 1 else chains.n_chains
    tau = np.full_like(q, np.nan)
    lp = np.ascontiguousarray(chains.link_ptr, dtype=np.int32)
    V0 = conv(np.zeros(6) if V0 is None else V0)
    dV0 = conv(oracle.GRAVITY_ACC if dV0 is None else dV0)
    fn(P, n_states, chains.n_chains, int(chains.lengths().max()), _p(lp), _p(conv(chains.placement)),
       _p(conv(chains.twist)), _p(conv(chains.inertia)), _p(q), _p(conv(st.qd)), _p(conv(st.qdd)), _p(tau),
       _p(conv(tip)), _p(V0), _p(dV0))
    return tau


def rel_rows(x, ref):
    return np.linalg.norm(x - ref, axis=-1) / np.linalg.norm(ref, axis=-1)


@pytest.mark.parametrize("P", [1, 2, 4, 8, 16, 32, 64])
def test_fp64_team_id_equals_serial_rnea(team_lib, P):
    """Every segment count, on a 13-link chain (segments of 13 down to 1 link, and empty ones), with base motion
    and a tip wrench: FP64 inverse dynamics equals the oracle's serial recursion to rounding."""
    ch = synth.make_chains([13], 41)
    st = synth.make_states((24, 13), 41)
    rng = np.random.default_rng(41)
    tip = rng.standard_normal((24, 6))
    V0, dV0 = rng.standard_normal(6), rng.standard_normal(6)
    tau = team_id(team_lib, P, ch, st, np.float64, tip, V0, dV0)
    for s in range(24):
        ref = oracle.rnea1(ch, st.q[s], st.qd[s], st.qdd[s], V0, dV0, tip[s])
        assert np.linalg.norm(tau[s] - ref) <= 1e-12 * np.linalg.norm(ref), (P, s)


@pytest.mark.parametrize("P", [1, 4, 8, 32])
def test_fp64_team_id_ragged(team_lib, P):
    ch = synth.make_chains([1, 2, 13, 5, 30, 64, 7], 43)
    st = synth.make_states((ch.n_links_total,), 43)
    tau = team_id(team_lib, P, ch, st, np.float64)
    ref = oracle.rnea(ch, st.q, st.qd, st.qdd)
    for c in range(ch.n_chains):
        a, b = ch.link_ptr[c], ch.link_ptr[c + 1]
        assert np.linalg.norm(tau[a:b] - ref[a:b]) <= 1e-12 * np.linalg.norm(ref[a:b]), (P, c)


@pytest.mark.parametrize("P", [1, 4, 16])
def test_fp32_team_id_100_links(team_lib, P):
    """FP32 bulk arithmetic with the wrench scan in FP64: per-state relative tau error within 1e-4 at 100 links."""
    ch, st = synth.make_chains([100], 45), synth.make_states((32, 100), 45)
    ch32, st32 = ch.astype(np.float32), st.astype(np.float32)
    tau = team_id(team_lib, P, ch32, st32, np.float32)
    chr_, str_ = ch.rounded(), st.rounded()
    ref = oracle.rnea(chr_, str_.q, str_.qd, str_.qdd)
    assert rel_rows(tau, ref).max() <= 1e-4


def team_fd(lib, P, chains, st, dtype, tip=None, V0=None, dV0=None):
    dt = np.dtype(dtype)
    fn = lib.cpu_team_fd_f64 if dt == np.float64 else lib.cpu_team_fd_f32
    conv = lambda a: None if a is None else np.ascontiguousarray(a, dtype=dt)
    q = conv(st.q)
    n_states = q.shape[0] if chains.n_chains == 1 else chains.n_chains
    qdd = np.full_like(q, np.nan)
    lp = np.ascontiguousarray(chains.link_ptr, dtype=np.int32)
    V0 = conv(np.zeros(6) if V0 is None else V0)
    dV0 = conv(oracle.GRAVITY_ACC if dV0 is None else dV0)
    faults = fn(P, n_states, chains.n_chains, int(chains.lengths().max()), _p(lp), _p(conv(chains.placement)),
                _p(conv(chains.twist)), _p(conv(chains.inertia)), _p(q), _p(conv(st.qd)), _p(conv(st.tau)), _p(qdd),
                _p(conv(tip)), _p(V0), _p(dV0))
    assert faults == 0
    return qdd


@pytest.mark.parametrize("P", [1, 2, 4, 8, 16])
def test_fp64_team_fd_equals_serial_aba(team_lib, P):
    """Forward dynamics with the bias forces by team scans and the serial articulated-body recursions,
    ragged chains (1 to 23 links), base motion and tip wrenches: equal to the oracle's ABA to rounding."""
    ch = synth.make_chains([13, 1, 23, 5, 8], 61)
    st = synth.make_states((ch.n_links_total,), 61)
    rng = np.random.default_rng(61)
    tip = rng.standard_normal((ch.n_chains, 6))
    V0, dV0 = rng.standard_normal(6), rng.standard_normal(6)
    qdd = team_fd(team_lib, P, ch, st, np.float64, tip=tip, V0=V0, dV0=dV0)
    ref = oracle.aba(ch, st.q, st.qd, st.tau, V0=V0, dV0=dV0, Ftip=tip)
    for c in range(ch.n_chains):
        a, b = ch.link_ptr[c], ch.link_ptr[c + 1]
        assert np.linalg.norm(qdd[a:b] - ref[a:b]) <= 1e-11 * np.linalg.norm(ref[a:b])


@pytest.mark.parametrize("P", [1, 8])
def test_fp32_team_fd_32_links(team_lib, P):
    """FP32, 32 links shared by 256 states: within the 1e-4 per-state bound of the FP32 path."""
    ch, st = synth.workload_32link(256)
    qdd = team_fd(team_lib, P, ch, st, np.float32)
    cr, sr = ch.rounded(), st.rounded()
    ref = oracle.aba(cr, sr.q, sr.qd, sr.tau)
    assert rel_rows(qdd.astype(np.float64), ref).max() <= 1e-4
