"""Pins of the oracle's shell spectrum and of the synthetic turbulence generator."""
import math

import numpy as np
import pytest
import torch

import synthetic
from oracle import spectrum


def test_single_mode_closed_form():
    # u_x = A sin(2 pi m x / n): the two Fourier coefficients +-m carry A/2 each,
    # so E(m) = 2 * 1/2 * (A/2)^2 = A^2/4 and all other shells are empty.
    n, m, A = 16, 3, 0.7
    x = torch.arange(n, dtype=torch.float64) * 2 * math.pi / n
    u = torch.zeros(3, n, n, n, dtype=torch.float64)
    u[0] = A * torch.sin(m * x)[None, None, :]
    E = spectrum.energy_spectrum(u)
    assert abs(float(E[m]) - A * A / 4) < 1e-15
    assert float(E.sum() - E[m]) < 1e-28


def test_parseval():
    u = synthetic.random_normal((3, 12, 10, 8), 81)
    E = spectrum.energy_spectrum(u)
    assert abs(float(E.sum()) / float(0.5 * (u * u).sum(0).mean()) - 1) < 1e-13


@pytest.mark.parametrize("dim,n", [(2, 32), (3, 24)])
def test_isotropic_generator(dim, n):
    k0, urms = 4.0, 0.05
    u = synthetic.isotropic_turbulence(n, k0, urms, seed=0, dim=dim)
    assert u.shape == (dim,) + (n,) * dim
    # rms per component and zero mean
    assert abs(math.sqrt(float((u * u).sum(0).mean()) / dim) - urms) < 1e-14
    assert float(u.mean(dim=tuple(range(1, dim + 1))).abs().max()) < 1e-17
    # spectrally divergence-free (central spectral derivative)
    uh = np.fft.fftn(u.numpy(), axes=tuple(range(1, dim + 1)))
    axes = np.meshgrid(*[np.fft.fftfreq(n, 1.0 / n)] * dim, indexing="ij")
    div = sum(axes[dim - 1 - a] * uh[a] for a in range(dim))
    assert np.abs(div).max() < 1e-12 * np.abs(uh).max() * n
    # shell spectrum proportional to K^4 exp(-2 (K/k0)^2) on every populated shell
    E = spectrum.energy_spectrum(u).numpy()
    K = np.arange(E.size, dtype=np.float64)
    target = K ** 4 * np.exp(-2 * (K / k0) ** 2)
    ok = (K >= 1) & (K < n // 2) & (E > 0)
    ratio = E[ok] / target[ok]
    assert np.ptp(ratio) < 1e-10 * ratio.mean()
    # seeded: the same seed gives the same field, another seed a different one
    assert torch.equal(u, synthetic.isotropic_turbulence(n, k0, urms, seed=0, dim=dim))
    assert not torch.equal(u, synthetic.isotropic_turbulence(n, k0, urms, seed=1, dim=dim))


def test_log_spectrum_loss():
    E = torch.tensor([0.0, 1e-3, 2e-3, 1e-9], dtype=torch.float64)
    T = torch.tensor([0.0, 1e-3, 1e-3, 1e-3], dtype=torch.float64)
    L = spectrum.log_spectrum_loss(E, T, 1, 3, 1e-6)
    assert abs(float(L) - (math.log(2.0) ** 2 + math.log(1e-6 / 1e-3) ** 2)) < 1e-12
