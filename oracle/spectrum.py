"""Energy spectrum and spectral loss (oracle side; test infrastructure).

The paper reports energy spectra E[k] (Sec. 3.1, decaying turbulence) and builds its
flow-control cost on the instantaneous spectrum sigma(u) (Sec. 3.2) without defining
either.  Reading used here (the standard shell spectrum of periodic turbulence):

    u_hat(k) = FFT(u)(k) / N            (N = number of cells)
    E(K)     = sum over wavevectors k with K - 1/2 <= |k| < K + 1/2 of  1/2 |u_hat(k)|^2

with integer wavevectors k in [-n/2, n/2).  By Parseval, sum_K E(K) = 1/2 <|u|^2>.

The loss follows the shape of the Sec. 3.2 cost: squared differences of the
logarithms of the spectra, each clipped from below at a cut-off c.
"""
from __future__ import annotations

import math

import torch


def wavenumber_magnitude(shape) -> torch.Tensor:
    """|k| on the FFT grid of a periodic box with the given spatial shape."""
    axes = [torch.fft.fftfreq(n, d=1.0 / n, dtype=torch.float64) for n in shape]
    mesh = torch.meshgrid(*axes, indexing="ij")
    return torch.sqrt(sum(m * m for m in mesh))


def shell_index(shape) -> torch.Tensor:
    """Integer shell K = floor(|k| + 1/2) of every wavevector."""
    return torch.floor(wavenumber_magnitude(shape) + 0.5).to(torch.int64)


def energy_spectrum(u: torch.Tensor) -> torch.Tensor:
    """E(K) for K = 0 .. K_max of a velocity field u[a, *spatial] (FP64)."""
    spatial = tuple(u.shape[1:])
    n_cells = math.prod(spatial)
    uh = torch.fft.fftn(u.to(torch.float64), dim=tuple(range(1, u.dim()))) / n_cells
    dens = 0.5 * (uh.real ** 2 + uh.imag ** 2).sum(dim=0)
    K = shell_index(spatial)
    E = torch.zeros(int(K.max()) + 1, dtype=torch.float64)
    return E.index_add(0, K.reshape(-1), dens.reshape(-1))


def log_spectrum_loss(E: torch.Tensor, E_target: torch.Tensor, k_lo: int, k_hi: int,
                      cutoff: float) -> torch.Tensor:
    """sum_{K=k_lo..k_hi} (ln max(E_K, c) - ln max(E_target_K, c))^2 (Sec. 3.2 cost,
    restricted to a band of shells)."""
    a = torch.log(torch.clamp(E[k_lo:k_hi + 1], min=cutoff))
    b = torch.log(torch.clamp(E_target[k_lo:k_hi + 1], min=cutoff))
    return ((a - b) ** 2).sum()
