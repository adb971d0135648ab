"""torch.autograd.Function over the library's integrations and their discrete adjoints.

ChemIntegrate maps (T0 [n], Y0 [ns, n], lnA [nr]) at pressure p [n] to (T_N [n], Y_N [ns, n]):
y0 = (T0, C(T0, p, Y0)) by the ideal-gas map, backward Euler over the split step (full Newton,
Section 3.2 of the paper) or the two-stage Rosenbrock method (Appendix A.3; adaptive, or fixed
steps with n_steps > 0), then Y_N = W C_N / rho.  The backward pass pulls the incoming gradients
back through the mass-fraction map, the recorded integration (discrete adjoint with checkpoint
recompute, deterministic reduction over cells for ln A; for Rosenbrock along the recorded
accepted steps) and the initial-state map -- all in the library's kernels.  Y0 is not
renormalised, so dL/dY0 are unconstrained partials.
"""

from __future__ import annotations

import torch

from ._binding import CHEM_BE, CHEM_PERSISTENT, CHEM_ROS2, Mechanism, Tape, default_options


class ChemIntegrate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, T0, Y0, lnA, mech: Mechanism, p, dt: float, n_steps: int, checkpoint_every: int = 50,
                energy: int = 0, method: int = CHEM_BE, max_steps: int = 4096):
        n = T0.shape[0]
        for t, shape in ((T0, (n,)), (Y0, (mech.ns, n)), (lnA, (mech.nr,)), (p, (n,))):
            if t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"expected a contiguous float64 CUDA tensor of shape {shape}")
        y = torch.empty((mech.n, n), dtype=torch.float64, device=T0.device)
        mech.chem_state_from_TPY(n, n, T0, p, Y0, y)
        if method == CHEM_ROS2:
            tape = Tape(mech, n, checkpoint_every, method=CHEM_ROS2, max_steps=max_steps)
        else:
            tape = Tape(mech, n, checkpoint_every)
        status = torch.empty(n, dtype=torch.int32, device=T0.device)
        opts = default_options(method=method, dt=dt, n_steps=n_steps, energy=energy, form=CHEM_PERSISTENT)
        mech.chem_integrate(n, n, y, lnA, opts, tape, status, None)
        YN = torch.empty((mech.ns, n), dtype=torch.float64, device=T0.device)
        mech.chem_mass_fractions(n, n, y, YN)
        TN = y[0].clone()
        ctx.save_for_backward(T0, Y0, p, y, lnA)
        ctx.mech, ctx.tape = mech, tape
        ctx.mark_non_differentiable(status)
        return TN, YN, status

    @staticmethod
    def backward(ctx, gTN, gYN, _gstatus):
        T0, Y0, p, yN, lnA = ctx.saved_tensors
        mech, tape = ctx.mech, ctx.tape
        n = T0.shape[0]
        dev = T0.device
        gTN = torch.zeros(n, dtype=torch.float64, device=dev) if gTN is None else gTN.contiguous()
        gYN = torch.zeros((mech.ns, n), dtype=torch.float64, device=dev) if gYN is None else gYN.contiguous()
        lamN = torch.empty((mech.n, n), dtype=torch.float64, device=dev)
        mech.chem_mass_fractions_vjp(n, n, yN, gYN, gTN, lamN)
        lam0 = torch.empty_like(lamN)
        glnA = torch.zeros(mech.nr, dtype=torch.float64, device=dev)
        mech.chem_integrate_adjoint(tape, lnA, lamN, lam0, glnA)
        dT0 = torch.empty(n, dtype=torch.float64, device=dev)
        dY0 = torch.empty((mech.ns, n), dtype=torch.float64, device=dev)
        mech.chem_state_from_TPY_vjp(n, n, T0, p, Y0, lam0, dT0, dY0)
        return dT0, dY0, glnA, None, None, None, None, None, None, None, None


def chem_integrate(T0, Y0, lnA, mech, p, dt, n_steps, checkpoint_every=50, energy=0, method=CHEM_BE,
                   max_steps=4096):
    """(T_N, Y_N, status) = one split step (backward Euler, or Rosenbrock with method=CHEM_ROS2 and at
    most max_steps recorded accepted steps per cell), differentiable in T0, Y0 and lnA."""
    return ChemIntegrate.apply(T0, Y0, lnA, mech, p, dt, n_steps, checkpoint_every, energy, method, max_steps)
