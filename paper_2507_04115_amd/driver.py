"""Spectral-phase parametrisation of the driving field, for gradients of a
harmonic-yield loss with respect to a few driver coefficients instead of
every field sample.

Every system's field is the same driver pulse seen at its own point of the
focus (amplitude and phase differ, the spectrum's support does not).  A
spectral phase phi(omega) common to all systems is added to each system's
spectrum:

    E_c(t) = irfft( rfft(E_0)(omega) * exp(i phi_c(omega)) ),
    phi_c(omega) = piecewise-linear interpolation of c_0 .. c_{m-1} placed
                   uniformly over the band where the batch's summed spectrum
                   exceeds `threshold` times its maximum (constant beyond
                   the end nodes).

c = 0 gives E_0 back.  The map is linear in exp(i phi), written with torch
FFTs, so torch autograd chains dl/dE from TDSEFunction (the adjoint kernel)
to dl/dc.  The paper drives its atoms with the field of its infrared
propagation; this parametrisation is the workload's optimisation knob, not
part of the paper's method.
"""
from __future__ import annotations

import torch

__all__ = ["SpectralPhase", "resample_field"]


class SpectralPhase:
    """phase = SpectralPhase(E0, n_nodes=64); E = phase(c)  (c: [n_nodes])."""

    def __init__(self, E0: torch.Tensor, n_nodes: int = 64, threshold: float = 1e-3):
        if E0.dim() != 2 or E0.dtype != torch.float64:
            raise TypeError("E0 must be a [systems, samples] float64 tensor")
        if n_nodes < 2:
            raise ValueError("n_nodes must be >= 2")
        self.n_samples = E0.shape[1]
        self.spec = torch.fft.rfft(E0.detach(), dim=1)
        mag = self.spec.abs().sum(dim=0)
        band = torch.nonzero(mag >= threshold * mag.max()).flatten()
        k_lo, k_hi = int(band.min()), int(band.max())
        if k_hi == k_lo:
            k_hi = k_lo + 1
        self.band = (k_lo, k_hi)
        self.n_nodes = n_nodes
        # interpolation weights [bins, nodes]: node j sits at bin
        # k_lo + j (k_hi - k_lo) / (n_nodes - 1)
        nb = self.spec.shape[1]
        u = (torch.arange(nb, dtype=torch.float64, device=E0.device) - k_lo) \
            * ((n_nodes - 1) / (k_hi - k_lo))
        u = u.clamp(0.0, n_nodes - 1)
        j0 = u.floor().long().clamp(max=n_nodes - 2)
        f = u - j0
        W = torch.zeros(nb, n_nodes, dtype=torch.float64, device=E0.device)
        rows = torch.arange(nb, device=E0.device)
        W[rows, j0] = 1.0 - f
        W[rows, j0 + 1] += f
        self.weights = W

    def phase(self, c: torch.Tensor) -> torch.Tensor:
        """phi_c at every rfft bin."""
        return self.weights @ c

    def __call__(self, c: torch.Tensor) -> torch.Tensor:
        if c.shape != (self.n_nodes,):
            raise ValueError(f"c must have shape ({self.n_nodes},)")
        phi = self.phase(c)
        rot = torch.polar(torch.ones_like(phi), phi)
        return torch.fft.irfft(self.spec * rot, n=self.n_samples, dim=1).contiguous()


def resample_field(e_coarse: torch.Tensor, dt_coarse: float, dt: float, nt: int) -> torch.Tensor:
    """Fields given at M coarse samples (spacing dt_coarse, the first sample
    taken as t = 0) resampled to E(i dt), i = 0..nt, by zero-padding their
    spectrum (section "1D-TSDE Implementation (CTDSE)": the input interface
    shifts the time axis to start at 0 and interpolates to dt in the Fourier
    domain).  The interpolant has period M dt_coarse, which must be an integer
    multiple M' >= max(M, nt + 1) of dt; for even M the Nyquist bin is split
    between +M/2 and -M/2.  Runs in the library (tdse_resample_field) on the
    tensor's device; the result is a contiguous [P, nt+1] float64 tensor
    ready for tdse_propagate_batch."""
    from . import binding as L

    e = torch.atleast_2d(e_coarse).to(torch.float64).contiguous()
    return L.tdse_resample_field(e, dt_coarse, dt, nt)
