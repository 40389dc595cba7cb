"""Seeded synthetic input fields shared by the oracle-side tests and the GPU path.

Holds no lattice-Boltzmann arithmetic: only the initial velocity/density fields and
random perturbations that both sides receive as inputs.  All fields are torch
float64 CPU tensors in the layout [component, (z,) y, x] with component 0 = x.

Workloads (the paper's flows, recreated as synthetic inputs):
  * Taylor-Green vortex in 2D and 3D (the benchmark flow of Sec. 3.3, the example of
    Listing 1).
  * Decaying isotropic turbulence (Sec. 3.1): a random-phase solenoidal field with a
    prescribed shell spectrum E(k) ~ k^4 exp(-2 (k/k0)^2), scaled to a target rms
    velocity per component.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def _axis(n: int) -> np.ndarray:
    """Cell-centre-free periodic coordinate x_i = 2 pi i / n."""
    return 2.0 * np.pi * np.arange(n, dtype=np.float64) / n


def taylor_green_2d(nx: int, ny: int, u0: float) -> torch.Tensor:
    """u = u0 (sin x cos y, -cos x sin y): returns [2, ny, nx]."""
    y, x = np.meshgrid(_axis(ny), _axis(nx), indexing="ij")
    u = np.stack([u0 * np.sin(x) * np.cos(y), -u0 * np.cos(x) * np.sin(y)])
    return torch.from_numpy(u)


def taylor_green_3d(nx: int, ny: int, nz: int, u0: float) -> torch.Tensor:
    """u = u0 (sin x cos y cos z, -cos x sin y cos z, 0): returns [3, nz, ny, nx]."""
    z, y, x = np.meshgrid(_axis(nz), _axis(ny), _axis(nx), indexing="ij")
    u = np.stack([u0 * np.sin(x) * np.cos(y) * np.cos(z),
                  -u0 * np.cos(x) * np.sin(y) * np.cos(z),
                  np.zeros_like(x)])
    return torch.from_numpy(u)


def _kvectors(shape):
    axes = [np.fft.fftfreq(n, d=1.0 / n) for n in shape]
    return np.meshgrid(*axes, indexing="ij")


def isotropic_turbulence(n: int, k0: float, u_rms: float, seed: int = 0, dim: int = 3) -> torch.Tensor:
    """Random-phase solenoidal velocity on an n^dim periodic box.

    Recipe: Gaussian white noise per component -> FFT -> remove the component along
    k (solenoidal projection) -> zero the mean and the Nyquist planes -> rescale each
    integer shell K = round(|k|) to E(K) ~ K^4 exp(-2 (K/k0)^2) -> inverse FFT ->
    scale so that sqrt(<u.u>/dim) = u_rms.  Returns [dim, (n,) n, n].
    """
    rng = np.random.default_rng(seed)
    shape = (n,) * dim
    noise = rng.standard_normal((dim,) + shape)
    uh = np.fft.fftn(noise, axes=tuple(range(1, dim + 1)))
    # Axis order of the spatial array is (z, y, x) / (y, x); wavevector component a
    # belongs to spatial axis dim-1-a.
    kax = _kvectors(shape)
    kvec = [kax[dim - 1 - a] for a in range(dim)]
    k2 = sum(k * k for k in kvec)
    k2_safe = np.where(k2 == 0, 1.0, k2)
    div = sum(kvec[a] * uh[a] for a in range(dim))
    for a in range(dim):
        uh[a] = uh[a] - kvec[a] * div / k2_safe
    nyq = np.zeros(shape, dtype=bool)
    for k in kvec:
        nyq |= np.abs(k) == n // 2
    mask = (k2 == 0) | nyq
    for a in range(dim):
        uh[a][mask] = 0.0
    kmag = np.sqrt(k2)
    shell = np.floor(kmag + 0.5).astype(np.int64)
    dens = 0.5 * (np.abs(uh) ** 2).sum(axis=0)
    e_now = np.bincount(shell.ravel(), weights=dens.ravel())
    K = np.arange(e_now.size, dtype=np.float64)
    e_target = K ** 4 * np.exp(-2.0 * (K / k0) ** 2)
    scale = np.zeros_like(e_now)
    ok = e_now > 0
    scale[ok] = np.sqrt(e_target[ok] / e_now[ok])
    uh = uh * scale[shell][None]
    u = np.real(np.fft.ifftn(uh, axes=tuple(range(1, dim + 1))))
    u -= u.mean(axis=tuple(range(1, dim + 1)), keepdims=True)
    rms = math.sqrt(float((u * u).sum(axis=0).mean()) / dim)
    u *= u_rms / rms
    return torch.from_numpy(np.ascontiguousarray(u))


def random_fields(spatial, dim: int, seed: int, drho: float = 0.05, umax: float = 0.08):
    """Uniform random density rho in [1-drho, 1+drho] and velocity components in
    [-umax, umax]: returns (rho [*spatial], u [dim, *spatial])."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + drho * (2.0 * rng.random(spatial) - 1.0)
    u = umax * (2.0 * rng.random((dim,) + tuple(spatial)) - 1.0)
    return torch.from_numpy(rho), torch.from_numpy(u)


def random_normal(shape, seed: int, scale: float = 1.0) -> torch.Tensor:
    """Seeded standard-normal array times scale (non-equilibrium perturbations,
    adjoint seeds, force fields, finite-difference directions)."""
    rng = np.random.default_rng(seed)
    return torch.from_numpy(scale * rng.standard_normal(shape))
