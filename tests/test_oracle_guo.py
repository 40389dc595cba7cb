"""Pins of the oracle's forced steps: the Guo body force (textbook; used by the
forced adjoint workloads) and the shifted-velocity equilibrium of the paper's flow
control (Sec. 3.2).

* Uniform body force: the physical momentum grows by exactly sum_x F per step.
* Kolmogorov flow F_x = F0 sin(k y): the steady state u_x = F0 sin(k y)/(rho nu k^2)
  is the exact Navier-Stokes solution (Krueger 2016, Sec. 6.5 uses this benchmark).
"""
import math

import torch

import synthetic
from oracle import lbm


def test_uniform_force_momentum_growth():
    st = lbm.stencil("D3Q27")
    spatial = (5, 6, 4)
    rho, u = synthetic.random_fields(spatial, 3, 31, drho=0.02, umax=0.03)
    F = torch.zeros((3,) + spatial, dtype=torch.float64)
    F[0] += 2e-5
    F[2] -= 1e-5
    g = lbm.equilibrium(rho, u, st)
    rho0, u0 = lbm.state_moments(g, st, F)
    P0 = (rho0 * u0).sum(dim=(1, 2, 3))
    total_F = F.sum(dim=(1, 2, 3))
    for t in range(1, 21):
        g = lbm.step(g, 0.7, st, F)
        r, v = lbm.state_moments(g, st, F)
        P = (r * v).sum(dim=(1, 2, 3))
        assert float((P - P0 - t * total_F).abs().max()) < 1e-12 * float(r.sum())


def test_kolmogorov_steady_state():
    st = lbm.stencil("D2Q9")
    nx, ny, tau = 4, 32, 0.8
    nu = lbm.nu_from_tau(tau)
    k = 2 * math.pi / ny
    umax = 0.01
    y = torch.arange(ny, dtype=torch.float64)
    F = torch.zeros(2, ny, nx, dtype=torch.float64)
    F[0] = (umax * nu * k * k * torch.sin(k * y))[:, None]
    g = lbm.equilibrium(torch.ones(ny, nx, dtype=torch.float64), torch.zeros(2, ny, nx, dtype=torch.float64), st)
    g = lbm.run(g, tau, st, 5000, F)
    r, v = lbm.state_moments(g, st, F)
    expect = umax * torch.sin(k * y)
    assert float((v[0, :, 0] - expect).abs().max()) < 1e-2 * umax
    assert float(v[1].abs().max()) < 1e-12


def test_forced_state_moments_match_literal_eq1():
    # Eq. 1 as printed, with the Guo force: f(t+1) = S(C(f(t))).  The stored state of
    # the pull convention is g(t) = C(f(t)); its moments must give rho(f(t)) and the
    # Guo velocity (sum c f(t) + F/2)/rho of the pre-collision state.
    st = lbm.stencil("D2Q9")
    spatial = (9, 11)
    rho, u = synthetic.random_fields(spatial, 2, 32, drho=0.02, umax=0.04)
    F = synthetic.random_normal((2,) + spatial, 33, 1e-3)
    tau = 0.62
    f = lbm.equilibrium(rho, u, st)
    g = lbm.bgk_collide(f, tau, st, F)
    for _ in range(10):
        r_g, u_g = lbm.state_moments(g, st, F)
        torch.testing.assert_close(r_g, lbm.density(f), rtol=1e-14, atol=0)
        torch.testing.assert_close(u_g, lbm.velocity(f, st, F), rtol=0, atol=1e-15)
        f = lbm.step_literal(f, tau, st, F)
        g = lbm.step(g, tau, st, F)


def test_shifted_equilibrium_momentum_gain():
    # f^eq(rho, u + du) has first moment rho (u + du) (Eq. 3's moments), so one
    # collision adds exactly rho du / tau of momentum and keeps the mass; du = 0 is
    # the plain BGK collision.
    for name, spatial in (("D2Q9", (6, 7)), ("D3Q19", (3, 4, 5)), ("D3Q27", (4, 3, 5))):
        st = lbm.stencil(name)
        rho, u = synthetic.random_fields(spatial, st.D, 34, drho=0.03, umax=0.05)
        f = lbm.equilibrium(rho, u, st) * (1 + synthetic.random_normal((st.Q,) + spatial, 35, 0.02))
        du = synthetic.random_normal((st.D,) + spatial, 36, 1e-3)
        tau = 0.58
        out = lbm.bgk_collide_shifted(f, tau, st, du)
        torch.testing.assert_close(lbm.density(out), lbm.density(f), rtol=1e-14, atol=0)
        gain = lbm.momentum(out, st) - lbm.momentum(f, st)
        torch.testing.assert_close(gain, lbm.density(f) * du / tau, rtol=0, atol=4e-16)  # FP64 roundoff
        zero = torch.zeros_like(du)
        torch.testing.assert_close(lbm.step_shifted(f, tau, st, zero), lbm.step(f, tau, st), rtol=0, atol=1e-16)
