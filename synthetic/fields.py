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


def taylor_green_2d_on(device, nx: int, ny: int, u0: float) -> torch.Tensor:
    """taylor_green_2d built directly on `device` by broadcasting (for grids too large
    to stage in host memory); the same field up to the last ulp of sin/cos."""
    x = torch.arange(nx, device=device, dtype=torch.float64) * (2 * math.pi / nx)
    y = torch.arange(ny, device=device, dtype=torch.float64) * (2 * math.pi / ny)
    u = torch.empty((2, ny, nx), device=device, dtype=torch.float64)
    u[0] = (u0 * torch.sin(x))[None, :] * torch.cos(y)[:, None]
    u[1] = (-u0 * torch.cos(x))[None, :] * torch.sin(y)[:, None]
    return u


def taylor_green_3d_on(device, nx: int, ny: int, nz: int, u0: float) -> torch.Tensor:
    """taylor_green_3d built directly on `device` by broadcasting (for grids too large
    to stage in host memory); the same field up to the last ulp of sin/cos."""
    x = torch.arange(nx, device=device, dtype=torch.float64) * (2 * math.pi / nx)
    y = torch.arange(ny, device=device, dtype=torch.float64) * (2 * math.pi / ny)
    z = torch.arange(nz, device=device, dtype=torch.float64) * (2 * math.pi / nz)
    u = torch.empty((3, nz, ny, nx), device=device, dtype=torch.float64)
    u[0] = ((u0 * torch.sin(x))[None, :] * torch.cos(y)[:, None])[None] * torch.cos(z)[:, None, None]
    u[1] = ((-u0 * torch.cos(x))[None, :] * torch.sin(y)[:, None])[None] * torch.cos(z)[:, None, None]
    u[2] = 0.0
    return u


def _kvectors(shape, device):
    axes = [torch.fft.fftfreq(n, d=1.0 / n, dtype=torch.float64, device=device) for n in shape]
    return torch.meshgrid(*axes, indexing="ij")


def isotropic_turbulence(n: int, k0: float, u_rms: float, seed: int = 0, dim: int = 3,
                         device="cpu") -> torch.Tensor:
    """Random-phase solenoidal velocity on an n^dim periodic box.

    Recipe: Gaussian white noise per component (numpy PCG64, the seed) -> FFT ->
    remove the component along k (solenoidal projection) -> zero the mean and the
    Nyquist planes -> rescale each integer shell K = floor(|k| + 1/2) to
    E(K) ~ K^4 exp(-2 (K/k0)^2) -> inverse FFT -> subtract the mean -> scale so that
    sqrt(<u.u>/dim) = u_rms.  Returns [dim, (n,) n, n] float64 on `device` (the FFTs
    run there; CPU and GPU results agree to FP64 roundoff).
    """
    rng = np.random.default_rng(seed)
    shape = (n,) * dim
    noise = torch.from_numpy(rng.standard_normal((dim,) + shape)).to(device)
    sp = tuple(range(1, dim + 1))
    uh = torch.fft.fftn(noise, dim=sp)
    del noise
    # Spatial axes are ordered (z, y, x) / (y, x): wavevector component a lives on
    # spatial axis dim-1-a.
    kax = _kvectors(shape, device)
    kvec = [kax[dim - 1 - a] for a in range(dim)]
    k2 = sum(k * k for k in kvec)
    k2_safe = torch.where(k2 == 0, torch.ones_like(k2), k2)
    div = sum(kvec[a] * uh[a] for a in range(dim))
    for a in range(dim):
        uh[a] -= kvec[a] * div / k2_safe
    del div
    mask = k2 == 0
    for k in kvec:
        mask |= k.abs() == n // 2
    uh[:, mask] = 0
    shell = torch.floor(torch.sqrt(k2) + 0.5).to(torch.int64)
    del k2, k2_safe, kvec, kax
    dens = 0.5 * (uh.real.square() + uh.imag.square()).sum(dim=0)
    e_now = torch.zeros(int(shell.max()) + 1, dtype=torch.float64, device=device)
    e_now.index_add_(0, shell.reshape(-1), dens.reshape(-1))
    del dens
    K = torch.arange(e_now.numel(), dtype=torch.float64, device=device)
    e_target = K ** 4 * torch.exp(-2.0 * (K / k0) ** 2)
    scale = torch.where(e_now > 0, torch.sqrt(e_target / torch.where(e_now > 0, e_now, torch.ones_like(e_now))),
                        torch.zeros_like(e_now))
    uh *= scale[shell][None]
    del shell
    u = torch.fft.ifftn(uh, dim=sp).real.contiguous()
    del uh
    u -= u.mean(dim=sp, keepdim=True)
    rms = math.sqrt(float((u * u).sum(dim=0).mean()) / dim)
    u *= u_rms / rms
    return u


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
