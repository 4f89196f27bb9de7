"""torch.autograd.Function wrappers over the HIP forward, adjoint and
harmonic-yield kernels.  They only marshal tensors into the C-ABI calls of
``binding``; the forward pass, the reverse (costate) sweep and the loss and
its gradient all run in libtdse.

    plan  = binding.Plan(params, n_per_system, adjoint_k=256)
    accel = TDSEFunction.apply(E, plan)                    # [P, nt+1]
    y     = HarmonicYield.apply(accel, dt, omega0, 21, 31) # [P]
    y.sum().backward()                                     # E.grad = d sum(y) / dE

The gradient is the exact discrete adjoint of the forward map (the paper
solves the forward problem only, section "1D-TSDE Implementation (CTDSE)"),
so it agrees with finite differences of the forward outputs to rounding.
The initial state is a constant of the map (no gradient with respect to
psi0).
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import binding as L

__all__ = ["TDSEFunction", "HarmonicYield", "TDSEBatch", "BandSpectrum", "FarFieldGeometry",
           "FarField"]


def _check_field(E: torch.Tensor, plan: "L.Plan"):
    if E.dtype != torch.float64 or not E.is_cuda:
        raise TypeError("E must be a float64 tensor on the GPU")
    if E.dim() != 2 or E.shape[0] != plan.batch or E.shape[1] != plan.params.nt + 1:
        raise ValueError(f"E must have shape [{plan.batch}, {plan.params.nt + 1}], "
                         f"got {tuple(E.shape)}")


class TDSEFunction(torch.autograd.Function):
    """accel = TDSEFunction.apply(E, plan, psi0=None).

    forward:  tdse_propagate_batch -> dipole acceleration [P, nt+1]
    backward: tdse_adjoint_batch with accel_bar = grad_output -> dl/dE
    The plan must have been created with adjoint_k > 0 for backward.  On a
    plan with TDSE_OPT_STORE_CHECKPOINTS, backward uses the checkpoints this
    forward stored (tdse_adjoint_batch_stored) while no later call has
    rewritten them, and recomputes the forward pass otherwise."""

    @staticmethod
    def forward(ctx, E: torch.Tensor, plan: "L.Plan", psi0: Optional[torch.Tensor] = None):
        _check_field(E, plan)
        E = E.contiguous()
        accel = torch.empty_like(E)
        L.tdse_propagate_batch(plan, E, psi0, accel)
        ctx.plan = plan
        ctx.psi0 = psi0
        ctx.generation = plan.checkpoint_generation() if plan.stores_checkpoints else 0
        ctx.save_for_backward(E)
        return accel

    @staticmethod
    def backward(ctx, grad_accel: torch.Tensor):
        (E,) = ctx.saved_tensors
        if ctx.plan.adjoint_k <= 0:
            raise RuntimeError("the plan was created without adjoint support (adjoint_k = 0)")
        grad_E = torch.empty_like(E)
        plan = ctx.plan
        if ctx.generation and plan.checkpoint_generation() == ctx.generation:
            L.tdse_adjoint_batch_stored(plan, ctx.generation, E, grad_accel.contiguous(), grad_E)
        else:
            L.tdse_adjoint_batch(plan, E, ctx.psi0, grad_accel.contiguous(), grad_E)
        return grad_E, None, None


class HarmonicYield(torch.autograd.Function):
    """y = HarmonicYield.apply(accel, dt, omega0, h_lo, h_hi): per-row Hann-
    windowed yield of harmonics h_lo..h_hi (tdse_harmonic_yield).  backward
    calls the same kernel with row_weight = grad_output, which returns
    grad_output[b] * d y[b] / d accel[b]."""

    @staticmethod
    def forward(ctx, accel: torch.Tensor, dt: float, omega0: float, h_lo: float, h_hi: float):
        if accel.dtype != torch.float64 or not accel.is_cuda or accel.dim() != 2:
            raise TypeError("accel must be a 2-D float64 tensor on the GPU")
        accel = accel.contiguous()
        batch, n1 = accel.shape
        _, nk = L.tdse_harmonic_band(n1 - 1, dt, omega0, h_lo, h_hi)
        work = torch.empty(2 * batch * max(nk, 1), dtype=torch.float64, device=accel.device)
        y = torch.empty(batch, dtype=torch.float64, device=accel.device)
        L.tdse_harmonic_yield(batch, n1 - 1, dt, omega0, h_lo, h_hi, accel, None, work, y)
        ctx.args = (dt, omega0, h_lo, h_hi)
        ctx.save_for_backward(accel)
        return y

    @staticmethod
    def backward(ctx, grad_y: torch.Tensor):
        (accel,) = ctx.saved_tensors
        dt, omega0, h_lo, h_hi = ctx.args
        batch, n1 = accel.shape
        _, nk = L.tdse_harmonic_band(n1 - 1, dt, omega0, h_lo, h_hi)
        work = torch.empty(2 * batch * max(nk, 1), dtype=torch.float64, device=accel.device)
        y = torch.empty(batch, dtype=torch.float64, device=accel.device)
        abar = torch.empty_like(accel)
        L.tdse_harmonic_yield(batch, n1 - 1, dt, omega0, h_lo, h_hi, accel,
                              grad_y.contiguous(), work, y, abar)
        return abar, None, None, None, None


class TDSEBatch:
    """A batch of systems with a plan that supports the adjoint:
    ``TDSEBatch(params, n_per)(E)`` is TDSEFunction.apply(E, plan)."""

    def __init__(self, params: "L.tdse_params", n_per_system: Sequence[int], adjoint_k: int = 256,
                 options: int = 0, store_checkpoints: bool = False):
        if store_checkpoints:
            options |= L.TDSE_OPT_STORE_CHECKPOINTS
        self.plan = L.Plan(params, n_per_system, options=options, adjoint_k=adjoint_k)

    def __call__(self, E: torch.Tensor, psi0: Optional[torch.Tensor] = None) -> torch.Tensor:
        return TDSEFunction.apply(E, self.plan, psi0)

    def close(self):
        self.plan.close()


class BandSpectrum(torch.autograd.Function):
    """amp = BandSpectrum.apply(accel, dt, omega0, h_lo, h_hi): the windowed
    band spectrum A_k of every row (tdse_band_dft), complex128 [P, nk].
    backward: tdse_band_dft_adjoint."""

    @staticmethod
    def forward(ctx, accel: torch.Tensor, dt: float, omega0: float, h_lo: float, h_hi: float):
        if accel.dtype != torch.float64 or not accel.is_cuda or accel.dim() != 2:
            raise TypeError("accel must be a 2-D float64 tensor on the GPU")
        accel = accel.contiguous()
        batch, n1 = accel.shape
        _, nk = L.tdse_harmonic_band(n1 - 1, dt, omega0, h_lo, h_hi)
        amp = torch.empty(batch, max(nk, 1), dtype=torch.complex128, device=accel.device)
        L.tdse_band_dft(batch, n1 - 1, dt, omega0, h_lo, h_hi, accel, amp)
        ctx.args = (batch, n1, dt, omega0, h_lo, h_hi)
        return amp[:, :nk]

    @staticmethod
    def backward(ctx, grad_amp: torch.Tensor):
        batch, n1, dt, omega0, h_lo, h_hi = ctx.args
        abar = torch.empty(batch, n1, dtype=torch.float64, device=grad_amp.device)
        L.tdse_band_dft_adjoint(batch, n1 - 1, dt, omega0, h_lo, h_hi,
                                grad_amp.to(torch.complex128).contiguous(), abar)
        return abar, None, None, None, None


class FarFieldGeometry:
    """Source grid (rho'_i, z'_j; source p = i * n_z + j), quadrature weights
    of rho' drho' dz' times the density, wave numbers of the band bins, and
    the observation points (rho_m at distance z_obs), as float64 tensors on
    the GPU."""

    def __init__(self, rho_src, z_src, weights, kwave, rho_obs, z_obs: float, device="cuda:0"):
        t = lambda x: torch.as_tensor(x, dtype=torch.float64, device=device).contiguous()
        self.rho_src, self.z_src, self.weights = t(rho_src), t(z_src), t(weights).reshape(-1)
        self.kwave, self.rho_obs = t(kwave), t(rho_obs)
        self.z_obs = float(z_obs)
        if self.weights.numel() != self.rho_src.numel() * self.z_src.numel():
            raise ValueError("weights must have n_rho * n_z entries")


class FarField(torch.autograd.Function):
    """field = FarField.apply(amp, geometry): the far field [n_obs, nk]
    (complex128) of the source spectra amp [n_rho n_z, nk] (tdse_far_field);
    backward: tdse_far_field_adjoint."""

    @staticmethod
    def forward(ctx, amp: torch.Tensor, geom: FarFieldGeometry):
        amp = amp.to(torch.complex128).contiguous()
        nk = geom.kwave.numel()
        if amp.shape != (geom.weights.numel(), nk):
            raise ValueError(f"amp must have shape [{geom.weights.numel()}, {nk}]")
        field = torch.empty(geom.rho_obs.numel(), nk, dtype=torch.complex128, device=amp.device)
        L.tdse_far_field(geom.rho_src, geom.z_src, geom.weights, geom.kwave, amp, geom.rho_obs,
                         geom.z_obs, field)
        ctx.geom = geom
        return field

    @staticmethod
    def backward(ctx, grad_field: torch.Tensor):
        geom = ctx.geom
        amp_bar = torch.empty(geom.weights.numel(), geom.kwave.numel(), dtype=torch.complex128,
                              device=grad_field.device)
        L.tdse_far_field(geom.rho_src, geom.z_src, geom.weights, geom.kwave,
                         grad_field.to(torch.complex128).contiguous(), geom.rho_obs, geom.z_obs,
                         amp_bar, adjoint=True)
        return amp_bar, None

