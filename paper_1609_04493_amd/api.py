"""Python binding of libpdyn (ctypes): argument marshalling only.

Every step of the dynamics runs in the HIP kernels of libpdyn.so; PyTorch
supplies device memory and the current stream. There is no CPU fallback: if
the library is not built, or a call fails, an exception is raised.
"""

from __future__ import annotations

import ctypes
import os
import threading

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdyn.so")

OP_RNEA_ID, OP_ABA_FD, OP_ID_FD, OP_RNEA_ID_VJP, OP_ABA_FD_VJP, OP_JSIIA_FD, OP_MASS_MATRIX = 0, 1, 2, 3, 4, 5, 6
OP_RNEA_ID_JACOBIAN, OP_ABA_FD_JACOBIAN, OP_RNEA_ID_HESSIAN, OP_ARTICULATED_INERTIA, OP_ABA_FD_SCAN = 7, 8, 9, 10, 11
GRAVITY_ACC = (0.0, 0.0, 9.81, 0.0, 0.0, 0.0)
ZERO6 = (0.0,) * 6


class PdynError(RuntimeError):
    pass


class _Model(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_int32), ("n_links_max", ctypes.c_int32), ("n_links_total", ctypes.c_int64),
                ("link_ptr", ctypes.c_void_p), ("placement", ctypes.c_void_p), ("twist", ctypes.c_void_p),
                ("inertia", ctypes.c_void_p), ("prepared", ctypes.c_void_p), ("order", ctypes.c_void_p),
                ("link_ptr_host", ctypes.c_void_p), ("order_host", ctypes.c_void_p)]


class _Batch(ctypes.Structure):
    _fields_ = [("n_states", ctypes.c_int32), ("base_vel", ctypes.c_double * 6), ("base_acc", ctypes.c_double * 6),
                ("tip_wrench", ctypes.c_void_p), ("block_threads", ctypes.c_int32), ("max_blocks", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("segments", ctypes.c_int32)]


_lib = None
_lib_lock = threading.Lock()

# name -> number of pointer arguments between (model, batch) and (workspace, bytes, stream)
_ENTRY_ARITY = {
    "pdyn_rnea_id": 4, "pdyn_aba_fd": 4, "pdyn_id_fd": 6,
    "pdyn_rnea_id_vjp": 8, "pdyn_aba_fd_vjp": 8,
    "pdyn_jsiia_fd": 4, "pdyn_mass_matrix": 2,
    "pdyn_rnea_id_jacobian": 6, "pdyn_aba_fd_jacobian": 6,
    "pdyn_rnea_id_hessian": 7,
    "pdyn_articulated_inertia": 2, "pdyn_aba_fd_scan": 4,
}


def lib():
    """Load libpdyn.so (built by paper_1609_04493_amd.build); raise if it is missing."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise PdynError(f"{LIB_PATH} is not built; run paper_1609_04493_amd.build.build() first")
            L = ctypes.CDLL(LIB_PATH)
            vp = ctypes.c_void_p
            for base, k in _ENTRY_ARITY.items():
                for name in (base, base + "_f64"):
                    if hasattr(L, name):
                        fn = getattr(L, name)
                        fn.argtypes = [ctypes.POINTER(_Model), ctypes.POINTER(_Batch)] + [vp] * k + [vp, ctypes.c_size_t, vp]
                        fn.restype = ctypes.c_int
            L.pdyn_workspace_bytes.argtypes = [ctypes.c_int, ctypes.POINTER(_Model), ctypes.POINTER(_Batch), ctypes.c_int]
            L.pdyn_workspace_bytes.restype = ctypes.c_size_t
            L.pdyn_strerror.argtypes = [ctypes.c_int]
            L.pdyn_strerror.restype = ctypes.c_char_p
            L.pdyn_max_links.restype = ctypes.c_int
            L.pdyn_launch_choice.argtypes = [ctypes.c_int, ctypes.POINTER(_Model), ctypes.POINTER(_Batch),
                                             ctypes.c_int] + [ctypes.POINTER(ctypes.c_int32)] * 4
            L.pdyn_launch_choice.restype = ctypes.c_int
            L.pdyn_load_tuning.argtypes = [ctypes.c_char_p]
            L.pdyn_load_tuning.restype = ctypes.c_int
            L.pdyn_model_prepared_bytes.argtypes = [ctypes.POINTER(_Model), ctypes.c_int]
            L.pdyn_model_prepared_bytes.restype = ctypes.c_size_t
            L.pdyn_model_prepare.argtypes = [ctypes.POINTER(_Model), ctypes.c_int, vp, ctypes.c_size_t, vp]
            L.pdyn_model_prepare.restype = ctypes.c_int
            ci, cd = ctypes.c_int, ctypes.c_double
            for name in ("pdyn_rollout", "pdyn_rollout_f64"):
                getattr(L, name).argtypes = [ctypes.POINTER(_Model), ctypes.POINTER(_Batch), ci, cd, ci] + [vp] * 5 + [vp, ctypes.c_size_t, vp]
                getattr(L, name).restype = ci
            for name in ("pdyn_rollout_vjp", "pdyn_rollout_vjp_f64"):
                getattr(L, name).argtypes = [ctypes.POINTER(_Model), ctypes.POINTER(_Batch), ci, cd, ci] + [vp] * 9 + [vp, ctypes.c_size_t, vp]
                getattr(L, name).restype = ci
            L.pdyn_rollout_workspace_bytes.argtypes = [ci, ctypes.POINTER(_Model), ctypes.POINTER(_Batch), ci, ci]
            L.pdyn_rollout_workspace_bytes.restype = ctypes.c_size_t
            L.pdyn_id_fd_noalloc.argtypes = [ctypes.POINTER(_Model), ctypes.POINTER(_Batch)] + [vp] * 7 + [vp]
            L.pdyn_id_fd_noalloc.restype = ctypes.c_int
            L.pdyn_read_status.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_uint32)]
            L.pdyn_read_status.restype = ctypes.c_int
            i64 = ctypes.c_int64
            for name in ("pdyn_euler_step", "pdyn_euler_step_f64"):
                getattr(L, name).argtypes = [i64, cd, vp, vp, vp, vp]
                getattr(L, name).restype = ci
            for name in ("pdyn_euler_step_vjp", "pdyn_euler_step_vjp_f64"):
                getattr(L, name).argtypes = [i64, cd, vp, vp, vp, vp, vp, i64, vp, vp, vp]
                getattr(L, name).restype = ci
            _lib = L
    return _lib


# status bits of a workspace (see Workspace.read_status)
STATUS_NONFINITE = 1
STATUS_PIVOT = 2
STATUS_WAIT = 4


def read_status(device=None, workspace=None) -> int:
    """Status bits of the calls on `device` that used the default (or the given) workspace; clears them."""
    ws = workspace if workspace is not None else _workspace(device or "cuda")
    return ws.read_status()


def _check(status: int, what: str):
    if status != 0:
        raise PdynError(f"{what}: {lib().pdyn_strerror(status).decode()} ({status})")


class Model:
    """A chain set resident on one device.

    ``chains`` holds ``placement`` [L,7], ``twist`` [L,6], ``inertia`` [L,10]
    and ``link_ptr`` [n_chains+1] (numpy or torch). With one chain it is
    shared by every state; with several, state s uses chain s.
    """

    def __init__(self, chains, device="cuda", dtype=torch.float32, prepare=True):
        self.device = torch.device(device)
        self.dtype = dtype
        t = lambda a: torch.as_tensor(np.asarray(a), dtype=dtype).contiguous().to(self.device)
        self.placement = t(chains.placement)
        self.twist = t(chains.twist)
        self.inertia = t(chains.inertia)
        lp = np.ascontiguousarray(chains.link_ptr, dtype=np.int32)
        self.n_chains = len(lp) - 1
        self.lengths = np.diff(lp)
        self.n_links_max = int(self.lengths.max())
        self.n_links_total = int(lp[-1])
        self.link_ptr_host = lp
        self.link_ptr = torch.as_tensor(lp).to(self.device) if self.n_chains > 1 else None
        # longest chains first (stable): wavefronts of similar lengths, longest work dispatched first
        self.order_host = (np.ascontiguousarray(np.argsort(-self.lengths, kind="stable"), dtype=np.int32)
                           if self.n_chains > 1 else None)
        self.order = torch.as_tensor(self.order_host).to(self.device) if self.n_chains > 1 else None
        self.use_order = True
        self.prepared = None
        self._prepared_order = True
        if prepare:
            self.prepare()

    def c_struct(self, with_prepared=True) -> _Model:
        if with_prepared and self.prepared is not None and self._prepared_order != self.use_order:
            self.prepare()  # the tables of one chain per state are laid out for the lane order
        prep = self.prepared if with_prepared else None
        use_order = self.use_order and self.order is not None
        order = self.order if use_order else None
        per_chain = self.n_chains > 1
        return _Model(self.n_chains, self.n_links_max, self.n_links_total,
                      0 if self.link_ptr is None else self.link_ptr.data_ptr(),
                      self.placement.data_ptr(), self.twist.data_ptr(), self.inertia.data_ptr(),
                      0 if prep is None else prep.data_ptr(), 0 if order is None else order.data_ptr(),
                      self.link_ptr_host.ctypes.data if per_chain else 0,
                      self.order_host.ctypes.data if use_order else 0)

    @property
    def scalar_bytes(self) -> int:
        return 8 if self.dtype == torch.float64 else 4

    def prepare(self):
        """Derive the per-link tables once (pdyn_model_prepare) so calls skip that kernel."""
        L = lib()
        m = self.c_struct(with_prepared=False)
        nbytes = L.pdyn_model_prepared_bytes(ctypes.byref(m), self.scalar_bytes)
        if nbytes == 0:
            raise PdynError("pdyn_model_prepared_bytes: invalid model")
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        tab = buf[off:off + nbytes]
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(L.pdyn_model_prepare(ctypes.byref(m), self.scalar_bytes, tab.data_ptr(), nbytes, stream),
               "pdyn_model_prepare")
        self._prepared_buf = buf
        self.prepared = tab
        self._prepared_order = self.use_order
        return self

    def invalidate(self):
        """Drop the derived tables (call after changing placement, twist or inertia in place)."""
        self.prepared = None

    def state_shape(self, n_states: int):
        return (n_states, self.n_links_max) if self.n_chains == 1 else (self.n_links_total,)


# Explicit launch fields per operation: (block_threads, max_blocks, variant, segments); 0 = library default
# (or the library's tuning table, see autotune.apply).
_launch_override = {}


def set_launch(op: int, block_threads: int = 0, max_blocks: int = 0, variant: int = 0, segments: int = 0):
    _launch_override[op] = (int(block_threads), int(max_blocks), int(variant), int(segments))


def _batch_struct(n_states, base_vel, base_acc, tip, op=None):
    b = _Batch()
    b.n_states = n_states
    b.block_threads, b.max_blocks, b.variant, b.segments = _launch_override.get(op, (0, 0, 0, 0))
    for k in range(6):
        b.base_vel[k] = float(base_vel[k])
        b.base_acc[k] = float(base_acc[k])
    b.tip_wrench = 0 if tip is None else tip.data_ptr()
    return b


class Workspace:
    """Reusable device scratch: grows on demand, 256-byte aligned."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes + 256 or self.buf.device != device:
            # zeroed once: the first word of a workspace is the status word of the calls using it
            self.buf = torch.zeros(max(nbytes, 256) + 256, dtype=torch.uint8, device=device)
        off = (-self.buf.data_ptr()) % 256
        return self.buf[off:]

    def read_status(self) -> int:
        """Status bits (STATUS_NONFINITE, STATUS_PIVOT) of the calls that used this workspace since the
        last read; clears them. Synchronises the current stream."""
        if self.buf is None:
            return 0
        off = (-self.buf.data_ptr()) % 256
        bits = ctypes.c_uint32(0)
        stream = torch.cuda.current_stream(self.buf.device).cuda_stream
        _check(lib().pdyn_read_status(ctypes.c_void_p(self.buf.data_ptr() + off), ctypes.c_void_p(stream),
                                      ctypes.byref(bits)), "pdyn_read_status")
        return int(bits.value)


_default_ws = {}


def _workspace(device):
    device = torch.device(device)
    if device.type == "cuda" and device.index is None:
        device = torch.device("cuda", torch.cuda.current_device())
    key = (str(device), threading.get_ident())
    if key not in _default_ws:
        _default_ws[key] = Workspace()
    return _default_ws[key]


def _n_states(model: Model, q: torch.Tensor) -> int:
    if model.n_chains == 1:
        if q.dim() != 2 or q.shape[1] != model.n_links_max:
            raise PdynError(f"expected joint arrays [B, {model.n_links_max}], got {tuple(q.shape)}")
        return q.shape[0]
    if q.dim() != 1 or q.shape[0] != model.n_links_total:
        raise PdynError(f"expected ragged joint arrays [{model.n_links_total}], got {tuple(q.shape)}")
    return model.n_chains


def _prep(model, arrays):
    for a in arrays:
        if a is None:
            continue
        if a.device != model.device or a.dtype != model.dtype or not a.is_contiguous():
            raise PdynError("joint arrays must be contiguous, on the model's device, of the model's dtype")


def _call(name, op, model, n_states, ptrs, base_vel, base_acc, tip, workspace, segments=None, variant=None):
    L = lib()
    fn = getattr(L, name + ("_f64" if model.dtype == torch.float64 else ""))
    m = model.c_struct()
    b = _batch_struct(n_states, base_vel, base_acc, tip, op)
    if segments is not None:
        b.segments = int(segments)
    if variant is not None:
        b.variant = int(variant)
    scalar = model.scalar_bytes
    nbytes = L.pdyn_workspace_bytes(op, ctypes.byref(m), ctypes.byref(b), scalar)
    if nbytes == 0:
        raise PdynError(f"{name}: invalid model/batch for workspace query")
    ws = (workspace or _workspace(model.device)).get(nbytes, model.device)
    stream = torch.cuda.current_stream(model.device).cuda_stream
    st = fn(ctypes.byref(m), ctypes.byref(b), *[0 if p is None else p.data_ptr() for p in ptrs],
            ws.data_ptr(), ws.numel(), stream)
    _check(st, name)


class Plan:
    """One library call with its arguments marshalled once. Calling the plan launches the same operation on
    the same tensors again, on the stream that was current when the plan was made: the per-call Python
    work of the functions below (argument checks, the C structs, the workspace query) is done here once,
    for loops that repeat a call. The plan keeps the tensors it points to alive; changing the model's
    launch choice or its tables afterwards needs a new plan."""

    def __init__(self, name, op, model, n_states, ptrs, base_vel, base_acc, tip, workspace):
        L = lib()
        self.name = name
        self._fn = getattr(L, name + ("_f64" if model.dtype == torch.float64 else ""))
        self._m = model.c_struct()
        self._b = _batch_struct(n_states, base_vel, base_acc, tip, op)
        nbytes = L.pdyn_workspace_bytes(op, ctypes.byref(self._m), ctypes.byref(self._b), model.scalar_bytes)
        if nbytes == 0:
            raise PdynError(f"{name}: invalid model/batch for workspace query")
        self._ws = (workspace or _workspace(model.device)).get(nbytes, model.device)
        stream = torch.cuda.current_stream(model.device).cuda_stream
        self._keep = (model, tip) + tuple(ptrs)
        self._args = (ctypes.byref(self._m), ctypes.byref(self._b),
                      *[0 if p is None else p.data_ptr() for p in ptrs], self._ws.data_ptr(), self._ws.numel(), stream)

    def __call__(self):
        st = self._fn(*self._args)
        if st:
            _check(st, self.name)


def plan_id_fd(model: Model, q, qd, qdd_in, tau_in, base_vel=ZERO6, base_acc=GRAVITY_ACC, tip=None, out=None,
               workspace=None) -> Plan:
    """A Plan of id_fd on these tensors (outputs allocated here unless `out` gives them): plan() runs
    pdyn_id_fd again; plan.out is (tau_out, qdd_out)."""
    n_states = _n_states(model, q)
    _prep(model, (q, qd, qdd_in, tau_in, tip))
    tau_out, qdd_out = (torch.empty_like(q), torch.empty_like(q)) if out is None else out
    _prep(model, (tau_out, qdd_out))
    plan = Plan("pdyn_id_fd", OP_ID_FD, model, n_states, (q, qd, qdd_in, tau_in, tau_out, qdd_out), base_vel,
                base_acc, tip, workspace)
    plan.out = (tau_out, qdd_out)
    return plan


def rnea_id(model: Model, q, qd, qdd, base_vel=ZERO6, base_acc=GRAVITY_ACC, tip=None, out=None, workspace=None):
    """tau = ID(q, qd, qdd, V0, dV0, F_tip) for every state (eq. (3))."""
    n_states = _n_states(model, q)
    _prep(model, (q, qd, qdd, tip))
    tau = torch.empty_like(q) if out is None else out
    _call("pdyn_rnea_id", OP_RNEA_ID, model, n_states, (q, qd, qdd, tau), base_vel, base_acc, tip, workspace)
    return tau


def aba_fd(model: Model, q, qd, tau, base_vel=ZERO6, base_acc=GRAVITY_ACC, tip=None, out=None, workspace=None):
    """qdd = FD(q, qd, tau, V0, dV0, F_tip) for every state (eq. (4))."""
    n_states = _n_states(model, q)
    _prep(model, (q, qd, tau, tip))
    qdd = torch.empty_like(q) if out is None else out
    _call("pdyn_aba_fd", OP_ABA_FD, model, n_states, (q, qd, tau, qdd), base_vel, base_acc, tip, workspace)
    return qdd


def id_fd(model: Model, q, qd, qdd_in, tau_in, base_vel=ZERO6, base_acc=GRAVITY_ACC, tip=None, out=None,
          workspace=None):
    """(ID(q, qd, qdd_in), FD(q, qd, tau_in)) of the same states in one pass."""
    n_states = _n_states(model, q)
    _prep(model, (q, qd, qdd_in, tau_in, tip))
    tau_out, qdd_out = (torch.empty_like(q), torch.empty_like(q)) if out is None else out
    _call("pdyn_id_fd", OP_ID_FD, model, n_states, (q, qd, qdd_in, tau_in, tau_out, qdd_out),
          base_vel, base_acc, tip, workspace)
    return tau_out, qdd_out


def jsiia_fd(model: Model, q, qd, tau, base_vel=ZERO6, base_acc=GRAVITY_ACC, tip=None, out=None, workspace=None):
    """qdd = M(q)^-1 (tau - tau_bias) by the joint-space inertia and its Cholesky factor (eq. (6)); shared chain."""
    n_states = _n_states(model, q)
    _prep(model, (q, qd, tau, tip))
    qdd = torch.empty_like(q) if out is None else out
    _call("pdyn_jsiia_fd", OP_JSIIA_FD, model, n_states, (q, qd, tau, qdd), base_vel, base_acc, tip, workspace)
    return qdd


def _jacobian(name, op, model, q, qd, x3, base_vel, base_acc, tip, out, workspace):
    n_states = _n_states(model, q)
    if model.n_chains != 1:
        raise PdynError(f"{name}: Jacobians need one chain shared by the batch")
    _prep(model, (q, qd, x3, tip))
    n = model.n_links_max
    if out is None:
        out = tuple(torch.empty((n_states, n, n), dtype=model.dtype, device=model.device) for _ in range(3))
    _call(name, op, model, n_states, (q, qd, x3) + tuple(out), base_vel, base_acc, tip, workspace)
    return out


def rnea_id_jacobian(model: Model, q, qd, qdd, base_vel=ZERO6, base_acc=GRAVITY_ACC, tip=None, out=None,
                     workspace=None):
    """(dtau/dq, dtau/dqd, dtau/dqdd = M), each [B, n, n], by pdyn_rnea_id_jacobian."""
    return _jacobian("pdyn_rnea_id_jacobian", OP_RNEA_ID_JACOBIAN, model, q, qd, qdd, base_vel, base_acc, tip, out,
                     workspace)


def aba_fd_jacobian(model: Model, q, qd, qdd, base_vel=ZERO6, base_acc=GRAVITY_ACC, tip=None, out=None,
                    workspace=None):
    """(dqdd/dq, dqdd/dqd, dqdd/dtau = M^-1), each [B, n, n], at qdd = FD(q, qd, tau), by pdyn_aba_fd_jacobian."""
    return _jacobian("pdyn_aba_fd_jacobian", OP_ABA_FD_JACOBIAN, model, q, qd, qdd, base_vel, base_acc, tip, out,
                     workspace)


HESSIAN_BLOCKS = ("q_q", "q_qd", "qd_qd", "q_qdd")


def rnea_id_hessian(model: Model, q, qd, qdd, blocks=HESSIAN_BLOCKS, base_vel=ZERO6, base_acc=GRAVITY_ACC, tip=None,
                    out=None, workspace=None):
    """Second derivatives of tau = ID(q, qd, qdd) by pdyn_rnea_id_hessian: a dict block -> [B, n, n, n] with
    H[s, i, j, k] = d^2 tau_i / dx_j dy_k for the requested blocks (x, y) in ("q_q", "q_qd", "qd_qd", "q_qdd");
    `out` may give the tensors for some blocks."""
    n_states = _n_states(model, q)
    if model.n_chains != 1:
        raise PdynError("pdyn_rnea_id_hessian: Hessians need one chain shared by the batch")
    if not blocks or any(b not in HESSIAN_BLOCKS for b in blocks):
        raise PdynError(f"pdyn_rnea_id_hessian: blocks must be a non-empty subset of {HESSIAN_BLOCKS}")
    _prep(model, (q, qd, qdd, tip))
    n = model.n_links_max
    res = dict(out or {})
    for b in blocks:
        if b not in res:
            res[b] = torch.empty((n_states, n, n, n), dtype=model.dtype, device=model.device)
    ptrs = tuple(res.get(b) if b in blocks else None for b in HESSIAN_BLOCKS)
    _call("pdyn_rnea_id_hessian", OP_RNEA_ID_HESSIAN, model, n_states, (q, qd, qdd) + ptrs, base_vel, base_acc, tip,
          workspace)
    return {b: res[b] for b in blocks}


def articulated_inertia(model: Model, q, segments=0, out=None, workspace=None):
    """Articulated-body inertias Jhat_i of eq. (7) for every state of a shared chain by
    pdyn_articulated_inertia: [B, n, 6, 6], Jhat[s, i] that of link i+1 in its own frame (twist (v, w) to
    wrench (f, n)). segments: lanes per state of the associative scan (a power of two 1..128; 1 = the serial
    recursion; 0 = the library's choice for this batch)."""
    n_states = _n_states(model, q)
    if model.n_chains != 1:
        raise PdynError("pdyn_articulated_inertia: needs one chain shared by the batch")
    _prep(model, (q,))
    n = model.n_links_max
    J = torch.empty((n_states, n, 6, 6), dtype=model.dtype, device=model.device) if out is None else out
    _call("pdyn_articulated_inertia", OP_ARTICULATED_INERTIA, model, n_states, (q, J), ZERO6, ZERO6, None,
          workspace, segments=segments)
    return J


def aba_fd_scan(model: Model, q, qd, tau, base_vel=ZERO6, base_acc=GRAVITY_ACC, tip=None, segments=0, out=None,
                workspace=None, split=False):
    """qdd = FD(q, qd, tau) of a shared chain by pdyn_aba_fd_scan: every recursion of the articulated-body
    algorithm as a prefix scan over `segments` lanes per state (a power of two 1..128; 0 = the library's
    choice). split: the bias wrench and z-hat as two scans instead of one merged scan. [B, n]."""
    n_states = _n_states(model, q)
    if model.n_chains != 1:
        raise PdynError("pdyn_aba_fd_scan: needs one chain shared by the batch")
    _prep(model, (q, qd, tau, tip))
    qdd = torch.empty_like(q) if out is None else out
    _prep(model, (qdd,))
    _call("pdyn_aba_fd_scan", OP_ABA_FD_SCAN, model, n_states, (q, qd, tau, qdd), base_vel, base_acc, tip,
          workspace, segments=segments, variant=2 if split else 0)
    return qdd


def mass_matrix(model: Model, q, out=None, workspace=None):
    """M(q) of eq. (17) for every state of a shared chain: [B, n, n]."""
    n_states = _n_states(model, q)
    _prep(model, (q,))
    n = model.n_links_max
    M = torch.empty((n_states, n, n), dtype=model.dtype, device=model.device) if out is None else out
    _call("pdyn_mass_matrix", OP_MASS_MATRIX, model, n_states, (q, M), ZERO6, ZERO6, None, workspace)
    return M


def id_fd_noalloc(model: Model, q, qd, qdd_in, tau_in, base_vel=ZERO6, base_acc=GRAVITY_ACC, tip=None, out=None,
                  status_out=None):
    """id_fd through pdyn_id_fd_noalloc: no workspace, the library's static device scratch instead.

    status_out: an int32 tensor of one element on the model's device that receives the call's status bits,
    or None."""
    if model.dtype != torch.float32:
        raise PdynError("id_fd_noalloc: FP32 only")
    n_states = _n_states(model, q)
    _prep(model, (q, qd, qdd_in, tau_in, tip))
    tau_out, qdd_out = (torch.empty_like(q), torch.empty_like(q)) if out is None else out
    m = model.c_struct()
    b = _batch_struct(n_states, base_vel, base_acc, tip, OP_ID_FD)
    stream = torch.cuda.current_stream(model.device).cuda_stream
    st = lib().pdyn_id_fd_noalloc(ctypes.byref(m), ctypes.byref(b), q.data_ptr(), qd.data_ptr(), qdd_in.data_ptr(),
                                  tau_in.data_ptr(), tau_out.data_ptr(), qdd_out.data_ptr(),
                                  None if status_out is None else status_out.data_ptr(), stream)
    _check(st, "pdyn_id_fd_noalloc")
    return tau_out, qdd_out


def _inertia_bar_like(model):
    n = model.n_links_max if model.n_chains == 1 else model.n_links_total
    return torch.empty((n, 10), dtype=model.dtype, device=model.device)


def rnea_id_vjp(model: Model, q, qd, qdd, tau_bar, base_vel=ZERO6, base_acc=GRAVITY_ACC, tip=None,
                want_inertia=True, out=None, workspace=None):
    """(q_bar, qd_bar, qdd_bar, inertia_bar) = (d tau/d(q, qd, qdd, pi))^T tau_bar."""
    n_states = _n_states(model, q)
    _prep(model, (q, qd, qdd, tau_bar, tip))
    if out is None:
        out = (torch.empty_like(q), torch.empty_like(q), torch.empty_like(q),
               _inertia_bar_like(model) if want_inertia else None)
    qb, qdb, qddb, pib = out
    _call("pdyn_rnea_id_vjp", OP_RNEA_ID_VJP, model, n_states, (q, qd, qdd, tau_bar, qb, qdb, qddb, pib),
          base_vel, base_acc, tip, workspace)
    return qb, qdb, qddb, pib


def aba_fd_vjp(model: Model, q, qd, qdd, qdd_bar, base_vel=ZERO6, base_acc=GRAVITY_ACC, tip=None,
               want_inertia=True, out=None, workspace=None):
    """(q_bar, qd_bar, tau_bar, inertia_bar) of qdd = FD(q, qd, tau) at its output qdd."""
    n_states = _n_states(model, q)
    _prep(model, (q, qd, qdd, qdd_bar, tip))
    if out is None:
        out = (torch.empty_like(q), torch.empty_like(q), torch.empty_like(q),
               _inertia_bar_like(model) if want_inertia else None)
    qb, qdb, tb, pib = out
    _call("pdyn_aba_fd_vjp", OP_ABA_FD_VJP, model, n_states, (q, qd, qdd, qdd_bar, qb, qdb, tb, pib),
          base_vel, base_acc, tip, workspace)
    return qb, qdb, tb, pib


def n_checkpoints(steps: int, every: int) -> int:
    return (steps + every - 1) // every


def _rollout_call(name, with_grad, model, n_states, steps, dt, every, ptrs, base_vel, base_acc, workspace):
    L = lib()
    fn = getattr(L, name + ("_f64" if model.dtype == torch.float64 else ""))
    m = model.c_struct()
    b = _batch_struct(n_states, base_vel, base_acc, None)
    nbytes = L.pdyn_rollout_workspace_bytes(with_grad, ctypes.byref(m), ctypes.byref(b), every, model.scalar_bytes)
    if nbytes == 0:
        raise PdynError(f"{name}: invalid arguments for workspace query")
    ws = (workspace or _workspace(model.device)).get(nbytes, model.device)
    stream = torch.cuda.current_stream(model.device).cuda_stream
    st = fn(ctypes.byref(m), ctypes.byref(b), int(steps), float(dt), int(every),
            *[0 if p is None else p.data_ptr() for p in ptrs], ws.data_ptr(), ws.numel(), stream)
    _check(st, name)


def rollout(model: Model, q0, qd0, tau_seq, dt, ckpt_every=10, base_vel=ZERO6, base_acc=GRAVITY_ACC,
            out=None, workspace=None):
    """Fused rollout (pdyn_rollout). Returns (q_T, qd_T, ckpt_q, ckpt_qd); tau_seq is [steps, *joint layout]."""
    n_states = _n_states(model, q0)
    steps = tau_seq.shape[0]
    _prep(model, (q0, qd0, tau_seq))
    C = n_checkpoints(steps, ckpt_every)
    if out is None:
        out = (q0.clone(), qd0.clone(), torch.empty((C,) + tuple(q0.shape), dtype=q0.dtype, device=q0.device),
               torch.empty((C,) + tuple(q0.shape), dtype=q0.dtype, device=q0.device))
    else:
        out[0].copy_(q0)
        out[1].copy_(qd0)
    q, qd, cq, cqd = out
    _rollout_call("pdyn_rollout", 0, model, n_states, steps, dt, ckpt_every, (tau_seq, q, qd, cq, cqd),
                  base_vel, base_acc, workspace)
    return q, qd, cq, cqd


def rollout_vjp(model: Model, tau_seq, ckpt_q, ckpt_qd, qT_bar, qdT_bar, dt, ckpt_every=10, base_vel=ZERO6,
                base_acc=GRAVITY_ACC, want_inertia=True, out=None, workspace=None):
    """Fused rollout adjoint (pdyn_rollout_vjp). Returns (q0_bar, qd0_bar, tau_bar_seq, inertia_bar)."""
    n_states = _n_states(model, qT_bar)
    steps = tau_seq.shape[0]
    _prep(model, (tau_seq, ckpt_q, ckpt_qd, qT_bar, qdT_bar))
    if out is None:
        out = (torch.empty_like(qT_bar), torch.empty_like(qT_bar), torch.empty_like(tau_seq),
               _inertia_bar_like(model) if want_inertia else None)
    q0b, qd0b, tb, pib = out
    _rollout_call("pdyn_rollout_vjp", 1, model, n_states, steps, dt, ckpt_every,
                  (tau_seq, ckpt_q, ckpt_qd, qT_bar, qdT_bar, q0b, qd0b, tb, pib), base_vel, base_acc, workspace)
    return q0b, qd0b, tb, pib


def _ptr(t):
    return None if t is None else t.data_ptr()


def euler_step(q, qd, qdd, dt):
    """In place: qd += dt qdd, then q += dt qd (pdyn_euler_step)."""
    for a in (q, qd, qdd):
        if a.dtype != q.dtype or a.device != q.device or not a.is_contiguous() or a.numel() != q.numel():
            raise PdynError("euler_step: q, qd, qdd must be contiguous, same size, dtype and device")
    name = "pdyn_euler_step" + ("_f64" if q.dtype == torch.float64 else "")
    stream = torch.cuda.current_stream(q.device).cuda_stream
    _check(getattr(lib(), name)(q.numel(), float(dt), q.data_ptr(), qd.data_ptr(), qdd.data_ptr(), stream), name)


def euler_step_vjp(q_bar, qd_bar, dt, qdd_bar=None, q_bar_fd=None, qd_bar_fd=None, pi_bar=None, pi_bar_fd=None):
    """Adjoint of euler_step, updating (q_bar, qd_bar) in place (pdyn_euler_step_vjp): first adds the later
    step's forward-dynamics cotangents (and pi_bar += pi_bar_fd), then, if qdd_bar is given, writes the
    cotangent of this step's qdd into it."""
    for a in (qd_bar, qdd_bar, q_bar_fd, qd_bar_fd):
        if a is not None and (a.dtype != q_bar.dtype or a.numel() != q_bar.numel() or not a.is_contiguous()):
            raise PdynError("euler_step_vjp: joint arrays must be contiguous, same size and dtype")
    n_pi = 0 if pi_bar is None else pi_bar.numel()
    name = "pdyn_euler_step_vjp" + ("_f64" if q_bar.dtype == torch.float64 else "")
    stream = torch.cuda.current_stream(q_bar.device).cuda_stream
    _check(getattr(lib(), name)(q_bar.numel(), float(dt), q_bar.data_ptr(), qd_bar.data_ptr(), _ptr(q_bar_fd),
                                _ptr(qd_bar_fd), _ptr(qdd_bar), n_pi, _ptr(pi_bar), _ptr(pi_bar_fd), stream), name)
