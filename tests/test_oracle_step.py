"""Pins of the oracle's full time step against closed forms and exact invariants.

* 2D Taylor-Green vortex: an exact Navier-Stokes solution whose amplitude decays as
  exp(-2 nu k^2 t) with nu = (tau - 1/2)/3 (Sec. 3.1's tau-nu relation); the values
  come from tests/golden/tgv2d_decay.json (closed form, see make_golden.py).
* 3D Taylor-Green vortex at small amplitude: viscous decay rate 3 nu k^2 of the
  velocity mode, converging at second order in the grid spacing.
* Eq. 1 taken literally (collide, then stream) against the pull convention the GPU
  path uses: identical moment trajectories from an equilibrium start.
* Mass and momentum conservation; the centre of mass moves by the total momentum.
"""
import json
import math
import os

import pytest
import torch

import synthetic
from oracle import lbm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tgv2d_decay.json")


def _tgv2d_amplitude(g, st, n, u0):
    _, v = lbm.state_moments(g, st)
    b = synthetic.taylor_green_2d(n, n, 1.0)[0]
    return float((v[0] * b).sum() / (b * b).sum()) / u0, float(0.5 * (v * v).sum())


def test_tgv2d_decay_matches_closed_form():
    gold = json.load(open(GOLDEN))
    st = lbm.stencil("D2Q9")
    n, u0, tau = gold["n"], gold["u0"], gold["tau"]
    u = synthetic.taylor_green_2d(n, n, u0)
    g = lbm.equilibrium(torch.ones(n, n, dtype=torch.float64), u, st)
    ke0 = float(0.5 * (u * u).sum())
    t_prev = 0
    for t, amp_ref, ke_ref in zip(gold["t"], gold["amplitude"], gold["energy_ratio"]):
        g = lbm.run(g, tau, st, t - t_prev)
        t_prev = t
        amp, ke = _tgv2d_amplitude(g, st, n, u0)
        assert abs(amp / amp_ref - 1) < gold["rel_tol"], (t, amp, amp_ref)
        assert abs(ke / ke0 / ke_ref - 1) < 2 * gold["rel_tol"], (t, ke / ke0, ke_ref)


def _tgv3d_rate_error(n, tau, u0=1e-3, t0=10, t1=50, lattice="D3Q27"):
    st = lbm.stencil(lattice)
    u = synthetic.taylor_green_3d(n, n, n, u0)
    g = lbm.equilibrium(torch.ones(n, n, n, dtype=torch.float64), u, st)
    b = u[0] / u0

    def amp(gg):
        _, v = lbm.state_moments(gg, st)
        return float((v[0] * b).sum() / (b * b).sum())

    g = lbm.run(g, tau, st, t0)
    a0 = amp(g)
    g = lbm.run(g, tau, st, t1 - t0)
    a1 = amp(g)
    rate = -math.log(a1 / a0) / (t1 - t0)
    k = 2 * math.pi / n
    return rate / (3 * lbm.nu_from_tau(tau) * k * k) - 1


@pytest.mark.parametrize("lattice", ["D3Q19", "D3Q27"])
def test_tgv3d_viscous_decay_second_order(lattice):
    e16 = _tgv3d_rate_error(16, 0.6, lattice=lattice)
    e32 = _tgv3d_rate_error(32, 0.6, lattice=lattice)
    assert abs(e32) < 0.01
    assert 3.0 < e16 / e32 < 5.0  # second-order convergence: halving dx quarters the error


@pytest.mark.parametrize("name,spatial", [("D2Q9", (12, 16)), ("D3Q19", (5, 6, 7)), ("D3Q27", (6, 5, 7))])
def test_literal_eq1_equals_pull_convention(name, spatial):
    st = lbm.stencil(name)
    rho, u = synthetic.random_fields(spatial, st.D, 21, drho=0.02, umax=0.05)
    f = lbm.equilibrium(rho, u, st)
    g = f.clone()
    tau = 0.7
    for _ in range(15):
        f = lbm.step_literal(f, tau, st)
        g = lbm.step(g, tau, st)
        r_f, u_f = lbm.density(f), lbm.momentum(f, st) / lbm.density(f)
        r_g, u_g = lbm.state_moments(g, st)
        torch.testing.assert_close(r_g, r_f, rtol=1e-13, atol=0)
        torch.testing.assert_close(u_g, u_f, rtol=0, atol=1e-14)


@pytest.mark.parametrize("name,spatial", [("D2Q9", (12, 16)), ("D3Q19", (5, 6, 7)), ("D3Q27", (6, 5, 7))])
def test_conservation_over_many_steps(name, spatial):
    st = lbm.stencil(name)
    rho, u = synthetic.random_fields(spatial, st.D, 22, drho=0.05, umax=0.05)
    g = lbm.equilibrium(rho, u, st) * (1 + synthetic.random_normal((st.Q,) + spatial, 23, 0.01))
    m0, j0 = float(g.sum()), lbm.momentum(g, st).sum(dim=tuple(range(1, st.D + 1)))
    g = lbm.run(g, 0.55, st, 100)
    assert abs(float(g.sum()) / m0 - 1) < 1e-13
    j1 = lbm.momentum(g, st).sum(dim=tuple(range(1, st.D + 1)))
    assert float((j1 - j0).abs().max()) < 1e-13 * m0


def test_centre_of_mass_moves_by_momentum():
    # A localised perturbation on a resting background (far from the periodic seam):
    # streaming moves every population by c_i, so sum_x x rho changes by sum_x rho u.
    st = lbm.stencil("D2Q9")
    n = 32
    rho = torch.ones(n, n, dtype=torch.float64)
    u = torch.zeros(2, n, n, dtype=torch.float64)
    rho[14:18, 13:19] += 0.01
    u[0, 14:18, 13:19] = 0.02
    u[1, 15:17, 14:18] = -0.01
    g = lbm.equilibrium(rho, u, st)
    y, x = torch.meshgrid(torch.arange(n, dtype=torch.float64), torch.arange(n, dtype=torch.float64), indexing="ij")
    for _ in range(4):
        r0 = lbm.density(g)
        J = lbm.momentum(g, st).sum(dim=(1, 2))
        g = lbm.step(g, 0.8, st)
        r1 = lbm.density(g)
        assert abs(float(((r1 - r0) * x).sum() - J[0])) < 1e-10  # roundoff of 1024 cells x 31
        assert abs(float(((r1 - r0) * y).sum() - J[1])) < 1e-10


def test_mrt_tgv2d_decay_follows_shear_relaxation_time():
    # With the MRT collision (Eq. 5) the shear viscosity comes from tau_3..5 alone
    # (Sec. 3.1: tau_n = nu/c_s^2 + 1/2); different ghost-moment times must leave the
    # Taylor-Green decay at the closed form of that viscosity.
    gold = json.load(open(GOLDEN))
    st = lbm.stencil("D2Q9")
    n, u0, tau = gold["n"], gold["u0"], gold["tau"]
    taus = [1.0, 1.0, 1.0, tau, tau, tau, 1.1, 1.3, 1.3]
    g = lbm.equilibrium(torch.ones(n, n, dtype=torch.float64), synthetic.taylor_green_2d(n, n, u0), st)
    for _ in range(gold["t"][-1]):
        g = lbm.step_mrt(g, taus, st)
    amp, _ = _tgv2d_amplitude(g, st, n, u0)
    assert abs(amp / gold["amplitude"][-1] - 1) < gold["rel_tol"]
