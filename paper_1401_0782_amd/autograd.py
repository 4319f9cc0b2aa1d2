"""torch.autograd.Function for T(E) of the real-space operator.

The differentiable input is the local potential V (N values).  The forward
pass builds the operator and calls negf_transmission; the backward pass calls
negf_transmission_grad with the incoming dL/dT(E) as energy weights, which
solves the adjoint systems with the same complex symmetric operator (A^T = A,
Eq. 6) and returns dL/dV.  Anything upstream of V (for example the depths of
Gaussian wells, V = -sum_a U_a phi_a) is differentiated by torch.
"""

from __future__ import annotations

import numpy as np
import torch

from . import api


class TransmissionFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V, geometry, energies, opts):
        """V: (N,) float64 tensor; geometry: object with nx, ny, nz, h, R,
        cap_left, cap_right and optional kb_* arrays; energies: 1-D array."""
        v = V.detach().to("cpu", torch.float64).numpy()
        op = api.negf_build_operator(geometry.nx, geometry.ny, geometry.nz, geometry.h,
                                     geometry.R, v, geometry.cap_left, geometry.cap_right,
                                     getattr(geometry, "kb_offsets", None),
                                     getattr(geometry, "kb_idx", None),
                                     getattr(geometry, "kb_val", None),
                                     getattr(geometry, "kb_energy", None))
        e = np.ascontiguousarray(energies, dtype=np.float64)
        T = api.negf_transmission(op, e, **(opts or {}))
        ctx.op = op
        ctx.energies = e
        ctx.opts = opts or {}
        ctx.device = V.device
        return torch.as_tensor(T, dtype=torch.float64, device=V.device)

    @staticmethod
    def backward(ctx, grad_T):
        w = grad_T.detach().to("cpu", torch.float64).numpy()
        opts = {k: v for k, v in ctx.opts.items() if k not in ("core", "col_begin", "col_count")}
        dV, _ = api.negf_transmission_grad(ctx.op, ctx.energies, w, want_T=False, **opts)
        ctx.op.close()
        return torch.as_tensor(dV, dtype=torch.float64, device=ctx.device), None, None, None


def transmission(V, geometry, energies, **opts):
    """T(E) as a differentiable function of the local potential V."""
    return TransmissionFn.apply(V, geometry, energies, opts)
