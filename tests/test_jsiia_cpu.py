"""The joint-space inertia kernel's passes (jsiia.hpp), compiled for the host, against the oracle (CPU only).

M(q) must equal the oracle's eq. (17) matrix (n inverse dynamics with unit
accelerations) to rounding, and the JSIIA forward dynamics must equal both the
oracle's JSIIA and its articulated-body FD. The kernel computes in double
after the joint angles' (sin, cos), so even the FP32 build is held close to
the FP64 oracle.
"""

import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1609_04493_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kernel_cpu", "jsiia_on_cpu.hip")


@pytest.fixture(scope="module")
def jlib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("jcpu") / "libjsiia_cpu.so")
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    extra = os.environ.get("PDYN_HOST_BUILD_FLAGS", "").split()  # set by the sanitizer run (test_sanitized_cpu)
    subprocess.run([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-host-only", *extra, "-o", out, SRC],
                   check=True)
    lib = ctypes.CDLL(out)
    for f in (lib.cpu_jsiia_f32, lib.cpu_jsiia_f64):
        f.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p] * 9
        f.restype = ctypes.c_int
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def run(lib, fd, ch, q, qd, tau, dtype):
    dt = np.dtype(dtype)
    fn = lib.cpu_jsiia_f64 if dt == np.float64 else lib.cpu_jsiia_f32
    c = lambda a: np.ascontiguousarray(a, dtype=dt)
    q = c(q)
    B, n = q.shape
    out = np.zeros((B, n, n) if not fd else (B, n), dt)
    bad = fn(int(fd), B, n, _p(c(ch.placement)), _p(c(ch.twist)), _p(c(ch.inertia)), _p(q),
             _p(c(qd) if fd else None), _p(c(tau) if fd else None), _p(out), _p(c(np.zeros(6))),
             _p(c(oracle.GRAVITY_ACC)))
    return out, bad


@pytest.mark.parametrize("n", [1, 7, 32])
def test_mass_matrix_equals_eq17_fp64(jlib, n):
    ch = synth.make_chains([n], 11 + n)
    st = synth.make_states((16, n), 11 + n)
    M, _ = run(jlib, False, ch, st.q, None, None, np.float64)
    for s in range(16):
        ref = oracle.mass_matrix(ch, st.q[s])
        assert np.abs(M[s] - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.array_equal(M[s], M[s].T)


@pytest.mark.parametrize("n", [1, 7, 10, 32])
def test_jsiia_fd_equals_oracle_fp64(jlib, n):
    ch = synth.make_chains([n], 21 + n)
    st = synth.make_states((16, n), 21 + n)
    qdd, bad = run(jlib, True, ch, st.q, st.qd, st.tau, np.float64)
    assert bad == 0
    ref_j = np.stack([oracle.jsiia1(ch, st.q[s], st.qd[s], st.tau[s]) for s in range(16)])
    ref_a = oracle.aba(ch, st.q, st.qd, st.tau)
    rel = lambda x, r: (np.linalg.norm(x - r, axis=1) / np.linalg.norm(r, axis=1)).max()
    assert rel(qdd, ref_j) <= 1e-10
    assert rel(qdd, ref_a) <= 1e-10


def test_jsiia_fd_fp32_inputs_32_links(jlib):
    """FP32 inputs: the oracle runs on the same rounded inputs; the kernel's double arithmetic keeps
    the error far below the 1e-4 per-state bound even though M is formed and factored."""
    ch, st = synth.workload_32link(64)
    qdd, bad = run(jlib, True, ch, st.q, st.qd, st.tau, np.float32)
    assert bad == 0
    cr, sr = ch.rounded(), st.rounded()
    ref = oracle.aba(cr, sr.q, sr.qd, sr.tau)
    e = np.linalg.norm(qdd - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert e.max() <= 1e-4


def test_jsiia_reports_a_non_positive_pivot(jlib):
    """A link with negative mass makes M indefinite for some states: the solve reports it."""
    ch = synth.make_chains([4], 5)
    ch.inertia[2, 0] = -40.0
    st = synth.make_states((32, 4), 5)
    _, bad = run(jlib, True, ch, st.q, st.qd, st.tau, np.float64)
    assert bad > 0
