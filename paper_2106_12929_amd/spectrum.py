"""Shell energy spectrum and log-spectrum loss on the GPU (torch.fft): the loss head
of the forcing-optimisation workload, differentiable by torch autograd.

Definitions (the paper names the spectrum sigma(u) and its log-deviation cost in
Sec. 3.2 without formulas; this is the standard reading): u_hat = FFT(u)/N over
the periodic box, E(K) = sum of 1/2 |u_hat(k)|^2 over integer wavevectors with
K - 1/2 <= |k| < K + 1/2; the loss sums (ln max(E, c) - ln max(E_target, c))^2 over
a band of shells.  Sums are taken in FP64.

The shell sums are segmented reductions over the wavevectors sorted by shell (a
permutation computed once per grid): no atomics, so the result is deterministic and
does not serialise on the few shell bins the way a scatter-add does.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch


@dataclass(frozen=True)
class Shells:
    """Wavevectors of a periodic grid grouped by shell K = floor(|k| + 1/2)."""

    spatial: tuple
    order: torch.Tensor    # flat wavevector indices sorted by shell
    lengths: torch.Tensor  # wavevectors per shell, K = 0 .. K_max
    shell: torch.Tensor    # shell of every flat wavevector


def shell_index(spatial, device) -> Shells:
    ks = [torch.fft.fftfreq(n, d=1.0 / n, device=device, dtype=torch.float64) for n in spatial]
    grids = torch.meshgrid(*ks, indexing="ij")
    kmag = torch.sqrt(sum(g * g for g in grids))
    shell = torch.floor(kmag + 0.5).to(torch.int64).reshape(-1)
    order = torch.argsort(shell, stable=True)
    lengths = torch.bincount(shell)
    return Shells(tuple(spatial), order, lengths, shell)


def energy_spectrum(u: torch.Tensor, shells: Shells | None = None) -> torch.Tensor:
    """E(K), K = 0..K_max, of u[a, *spatial] (promoted to FP64)."""
    spatial = tuple(u.shape[1:])
    if shells is None:
        shells = shell_index(spatial, u.device)
    uh = torch.fft.fftn(u.to(torch.float64), dim=tuple(range(1, u.dim()))) / math.prod(spatial)
    dens = 0.5 * (uh.real.square() + uh.imag.square()).sum(dim=0)
    return torch.segment_reduce(dens.reshape(-1)[shells.order], "sum", lengths=shells.lengths, unsafe=True)


def log_spectrum_loss(E: torch.Tensor, E_target: torch.Tensor, k_lo: int, k_hi: int, cutoff: float) -> torch.Tensor:
    a = torch.log(torch.clamp(E[k_lo:k_hi + 1], min=cutoff))
    b = torch.log(torch.clamp(E_target[k_lo:k_hi + 1], min=cutoff))
    return (a - b).square().sum()


def log_spectrum_loss_and_grad(u: torch.Tensor, shells: Shells, E_target: torch.Tensor, k_lo: int, k_hi: int,
                               cutoff: float):
    """log_spectrum_loss(energy_spectrum(u), ...) and its gradient with respect to u,
    without autograd.  With u_hat = FFT(u)/N and g(k) = dR/dE_K at the shell K of k
    (2 (ln E_K - ln max(E_target, c)) / E_K inside the band where E_K >= c, else 0):
    dR/du = Re IFFT(g u_hat), since E_K sums 1/2 |u_hat|^2 and the FFT is linear.
    Two FFTs, a shell sum and a gather: the loss head of a controlled step."""
    spatial = tuple(u.shape[1:])
    dims = tuple(range(1, u.dim()))
    uh = torch.fft.fftn(u.to(torch.float64), dim=dims) / math.prod(spatial)
    dens = 0.5 * (uh.real.square() + uh.imag.square()).sum(dim=0)
    E = torch.segment_reduce(dens.reshape(-1)[shells.order], "sum", lengths=shells.lengths, unsafe=True)
    band = slice(k_lo, k_hi + 1)
    a = torch.log(torch.clamp(E[band], min=cutoff))
    b = torch.log(torch.clamp(E_target[band], min=cutoff))
    R = (a - b).square().sum()
    dE = torch.zeros_like(E)
    dE[band] = torch.where(E[band] >= cutoff, 2.0 * (a - b) / E[band], torch.zeros_like(a))
    g = dE[shells.shell].reshape(spatial)
    grad = torch.fft.ifftn(g * uh, dim=dims).real
    return R, grad


class NativeLossHead:
    """s * dR/du of R = log_spectrum_loss(energy_spectrum(u), E_target, k_lo, k_hi,
    cutoff), the quantity log_spectrum_loss_and_grad returns, computed by the library's
    kernels between two FFTs: FFT(u), lbm_shell_energy, lbm_log_spectrum_grad (which
    multiplies the coefficients by dR/dE at their shell and also writes R), inverse FFT,
    lbm_real_part.  Five launches beside the transforms, against about twenty torch
    launches; the shell sums take another fixed order, so the two agree to rounding."""

    def __init__(self, shells: Shells, E_target: torch.Tensor, k_lo: int, k_hi: int, cutoff: float):
        from . import binding

        self._B = binding
        self.table = binding.ShellTable.from_shells(shells.shell)
        if E_target.numel() != self.table.nshell:
            raise ValueError(f"E_target needs {self.table.nshell} shells (got {E_target.numel()})")
        self.E_target = E_target.to(torch.float64).contiguous()
        self.k_lo, self.k_hi, self.cutoff = int(k_lo), int(k_hi), float(cutoff)
        self.inv_n = 1.0 / math.prod(shells.spatial)
        self.E = torch.empty(self.table.nshell, dtype=torch.float64, device=E_target.device)
        self.R = torch.empty(1, dtype=torch.float64, device=E_target.device)

    def scaled_grad(self, u: torch.Tensor, scale: float, out: torch.Tensor, with_cost: bool = False) -> None:
        """out <- scale * dR/du for u[D, *spatial]; out float32 or float64 of u's shape.
        self.E holds the spectrum of u afterwards, and self.R its cost if with_cost."""
        dims = tuple(range(1, u.dim()))
        uh = torch.fft.fftn(u.to(torch.complex128), dim=dims)
        self._B.lbm_shell_energy(self.table, uh, self.inv_n, self.E)
        # the inverse transform's 1/N is folded into the multiplier: norm="forward"
        # leaves the inverse unscaled, which saves torch's separate scaling launch
        self._B.lbm_log_spectrum_grad(self.table, uh, self.E, self.E_target, self.k_lo, self.k_hi, self.cutoff,
                                      self.inv_n * self.inv_n, self.R if with_cost else None)
        self._B.lbm_real_part(torch.fft.ifftn(uh, dim=dims, norm="forward"), scale, out)
