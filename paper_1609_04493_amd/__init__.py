"""pdyn: batched rigid-body dynamics of serial chains on MI355X (gfx950).

Scan-form recursive Newton-Euler inverse dynamics and articulated-body
forward dynamics after Yang, Wu & Pan (arXiv:1609.04493), as hand-written HIP
kernels behind the C ABI of include/pdyn.h. This package is the thin Python
binding; ``synth`` is the seeded input generator.
"""

from .api import (GRAVITY_ACC, STATUS_NONFINITE, STATUS_PIVOT, Model, PdynError, Workspace, aba_fd, aba_fd_vjp,
                  aba_fd_scan, articulated_inertia, id_fd, lib, read_status, rnea_id, rnea_id_vjp)
from .autograd import forward_dynamics, inverse_dynamics
from .jacobian import fd_jacobians, id_hessians, id_jacobians

__all__ = ["GRAVITY_ACC", "STATUS_NONFINITE", "STATUS_PIVOT", "Model", "PdynError", "Workspace", "aba_fd",
           "aba_fd_scan", "aba_fd_vjp", "articulated_inertia", "fd_jacobians", "forward_dynamics", "id_fd", "id_hessians", "id_jacobians", "inverse_dynamics", "lib",
           "read_status", "rnea_id", "rnea_id_vjp"]
