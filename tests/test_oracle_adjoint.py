"""Pins of the gradient oracle (autograd through the FP64 step) by central finite
differences: the transposition identity <lam, J dg> = <J^T lam, dg> with J dg taken
by finite differences, for the step, the forced step, the moments map and a whole
rollout with a spectral loss."""
import pytest
import torch

import synthetic
from oracle import adjoint, lbm, spectrum

CASES = [("D2Q9", (6, 5)), ("D3Q19", (3, 4, 5)), ("D3Q27", (4, 3, 5))]


def _fd(fun, x, dx, eps):
    return (fun(x + eps * dx) - fun(x - eps * dx)) / (2 * eps)


def _state(name, spatial, seed):
    st = lbm.stencil(name)
    rho, u = synthetic.random_fields(spatial, st.D, seed, drho=0.05, umax=0.08)
    g = lbm.equilibrium(rho, u, st) * (1 + synthetic.random_normal((st.Q,) + spatial, seed + 1, 0.02))
    return st, g


@pytest.mark.parametrize("name,spatial", CASES)
@pytest.mark.parametrize("forced", [False, True])
def test_step_vjp_transposition(name, spatial, forced):
    st, g = _state(name, spatial, 51)
    tau = 0.57
    F = synthetic.random_normal((st.D,) + spatial, 53, 1e-3) if forced else None
    lam = synthetic.random_normal((st.Q,) + spatial, 54)
    dg = synthetic.random_normal((st.Q,) + spatial, 55, 1e-2)
    vjp, dF = adjoint.step_vjp(g, lam, tau, st, F)
    jvp = _fd(lambda x: lbm.step(x, tau, st, F), g, dg, 1e-5)
    lhs, rhs = float((lam * jvp).sum()), float((vjp * dg).sum())
    assert abs(lhs - rhs) <= 1e-8 * abs(rhs)
    if forced:
        dFdir = synthetic.random_normal((st.D,) + spatial, 56, 1e-3)
        jvpF = _fd(lambda x: lbm.step(g, tau, st, x), F, dFdir, 1e-4)
        lhs, rhs = float((lam * jvpF).sum()), float((dF * dFdir).sum())
        assert abs(lhs - rhs) <= 1e-8 * abs(rhs)


@pytest.mark.parametrize("name,spatial", CASES)
@pytest.mark.parametrize("forced", [False, True])
def test_moments_vjp(name, spatial, forced):
    st, g = _state(name, spatial, 61)
    F = synthetic.random_normal((st.D,) + spatial, 62, 1e-3) if forced else None
    a = synthetic.random_normal(spatial, 63)
    b = synthetic.random_normal((st.D,) + spatial, 64)
    dg = synthetic.random_normal((st.Q,) + spatial, 65, 1e-2)
    vjp, dF = adjoint.moments_vjp(g, st, F, a, b)

    def fwd(x):
        r, u = lbm.state_moments(x, st, F)
        return (a * r).sum() + (b * u).sum()

    lhs = float(_fd(fwd, g, dg, 1e-5))
    rhs = float((vjp * dg).sum())
    assert abs(lhs - rhs) <= 1e-8 * abs(rhs)
    if forced:
        # u = (sum c g - F/2)/rho  =>  dL/dF = -b / (2 rho)
        torch.testing.assert_close(dF, -0.5 * b / lbm.density(g), rtol=1e-14, atol=0)


def test_rollout_grad_spectral_loss():
    st = lbm.stencil("D3Q27")
    n = 8
    u = synthetic.isotropic_turbulence(n, 2.0, 0.03, seed=3)
    g0 = lbm.equilibrium(torch.ones(n, n, n, dtype=torch.float64), u, st)
    F = synthetic.random_normal((3, n, n, n), 71, 1e-4)
    K = torch.arange(n, dtype=torch.float64).clamp(min=1)
    target = 1e-4 * K ** (-5.0 / 3.0)

    def loss(rho, uu):
        return spectrum.log_spectrum_loss(spectrum.energy_spectrum(uu), target, 1, 3, 1e-14)

    L, dg0, dF = adjoint.rollout_grad(g0, F, 0.6, st, 5, loss)
    dFdir = synthetic.random_normal((3, n, n, n), 72, 1e-4)

    def L_of_F(x):
        g = g0
        for _ in range(5):
            g = lbm.step(g, 0.6, st, x)
        r, v = lbm.state_moments(g, st, x)
        return loss(r, v)

    fd = float(_fd(L_of_F, F, dFdir, 1e-3))
    an = float((dF * dFdir).sum())
    assert abs(fd - an) <= 1e-6 * abs(an)
