"""Pins of the oracle's equilibrium (Eq. 3), moments (Eq. 4), BGK collision (Eq. 2)
and Guo forcing term.

Each check is a fact fixed by the mathematics rather than the formula retyped:
the second-order equilibrium reproduces the first three Maxwellian moments
exactly, collision conserves mass and momentum and fixes the equilibrium, and
the Guo source has known zeroth/first/second moments.
"""
import pytest
import torch

import synthetic
from oracle import lbm

CASES = [("D2Q9", (7, 5)), ("D3Q19", (3, 4, 5)), ("D3Q27", (4, 5, 3))]


def _state(name, spatial, seed):
    st = lbm.stencil(name)
    rho, u = synthetic.random_fields(spatial, st.D, seed, drho=0.1, umax=0.1)
    return st, rho, u


@pytest.mark.parametrize("name,spatial", CASES)
def test_equilibrium_moments(name, spatial):
    st, rho, u = _state(name, spatial, 1)
    feq = lbm.equilibrium(rho, u, st)
    cf = st.c.to(torch.float64)
    m0 = feq.sum(0)
    m1 = torch.einsum("qa,q...->a...", cf, feq)
    m2 = torch.einsum("qa,qb,q...->ab...", cf, cf, feq)
    torch.testing.assert_close(m0, rho, rtol=1e-14, atol=0)
    torch.testing.assert_close(m1, rho * u, rtol=1e-13, atol=1e-16)
    eye = torch.eye(st.D, dtype=torch.float64).reshape((st.D, st.D) + (1,) * len(spatial))
    expect = rho * (u[:, None] * u[None, :]) + rho * eye / 3.0
    torch.testing.assert_close(m2, expect, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("name,spatial", CASES)
def test_rest_equilibrium_is_weights(name, spatial):
    st = lbm.stencil(name)
    rho = torch.ones(spatial, dtype=torch.float64)
    u = torch.zeros((st.D,) + spatial, dtype=torch.float64)
    feq = lbm.equilibrium(rho, u, st)
    assert torch.equal(feq, st.w.reshape((st.Q,) + (1,) * len(spatial)).expand_as(feq))


@pytest.mark.parametrize("name,spatial", CASES)
@pytest.mark.parametrize("tau", [0.51, 0.6, 1.0, 1.7])
def test_equilibrium_fixed_point(name, spatial, tau):
    st, rho, u = _state(name, spatial, 2)
    feq = lbm.equilibrium(rho, u, st)
    out = lbm.bgk_collide(feq, tau, st)
    # a few FP64 ulps of populations of size <= 1
    assert float((out - feq).abs().max()) < 8 * 2.0 ** -52


@pytest.mark.parametrize("name,spatial", CASES)
@pytest.mark.parametrize("tau", [0.51, 0.8])
def test_collision_conserves_mass_momentum(name, spatial, tau):
    st, rho, u = _state(name, spatial, 3)
    f = lbm.equilibrium(rho, u, st) * (1.0 + synthetic.random_normal((st.Q,) + spatial, 4, 0.05))
    out = lbm.bgk_collide(f, tau, st)
    torch.testing.assert_close(lbm.density(out), lbm.density(f), rtol=1e-14, atol=0)
    torch.testing.assert_close(lbm.momentum(out, st), lbm.momentum(f, st), rtol=0, atol=1e-15)


@pytest.mark.parametrize("name,spatial", CASES)
def test_tau_one_gives_equilibrium(name, spatial):
    # Special case of Eq. 2: with tau = 1 collision replaces f by f^eq(rho(f), u(f)).
    st, rho, u = _state(name, spatial, 5)
    f = lbm.equilibrium(rho, u, st) * (1.0 + synthetic.random_normal((st.Q,) + spatial, 6, 0.05))
    out = lbm.bgk_collide(f, 1.0, st)
    feq = lbm.equilibrium(lbm.density(f), lbm.momentum(f, st) / lbm.density(f), st)
    torch.testing.assert_close(out, feq, rtol=0, atol=4e-16)


@pytest.mark.parametrize("name,spatial", CASES)
def test_nonequilibrium_part_relaxes_by_one_minus_omega(name, spatial):
    # BGK keeps the conserved moments, so f^eq of the collided state is f^eq of the
    # input; hence the non-equilibrium part shrinks by exactly (1 - 1/tau).
    st, rho, u = _state(name, spatial, 7)
    tau = 0.7
    f = lbm.equilibrium(rho, u, st) * (1.0 + synthetic.random_normal((st.Q,) + spatial, 8, 0.05))
    fe = lambda g: lbm.equilibrium(lbm.density(g), lbm.momentum(g, st) / lbm.density(g), st)
    out = lbm.bgk_collide(f, tau, st)
    torch.testing.assert_close(out - fe(out), (1 - 1 / tau) * (f - fe(f)), rtol=0, atol=2e-16)


@pytest.mark.parametrize("name,spatial", CASES)
def test_guo_source_moments(name, spatial):
    # Guo et al. 2002: sum S = 0, sum c S = (1 - 1/2tau) F,
    # sum c_a c_b S = (1 - 1/2tau)(u_a F_b + u_b F_a).
    st, rho, u = _state(name, spatial, 9)
    F = synthetic.random_normal((st.D,) + spatial, 10, 1e-3)
    tau = 0.65
    S = lbm.guo_source(u, F, tau, st)
    cf = st.c.to(torch.float64)
    k = 1 - 0.5 / tau
    torch.testing.assert_close(S.sum(0), torch.zeros(spatial, dtype=torch.float64), rtol=0, atol=1e-18)
    torch.testing.assert_close(torch.einsum("qa,q...->a...", cf, S), k * F, rtol=1e-13, atol=1e-19)
    m2 = torch.einsum("qa,qb,q...->ab...", cf, cf, S)
    expect = k * (u[:, None] * F[None, :] + u[None, :] * F[:, None])
    torch.testing.assert_close(m2, expect, rtol=1e-12, atol=1e-19)


@pytest.mark.parametrize("name,spatial", CASES)
def test_forced_collision_momentum_gain(name, spatial):
    # With the Guo scheme, collision adds exactly F to sum_i c_i f_i and keeps rho.
    st, rho, u = _state(name, spatial, 11)
    F = synthetic.random_normal((st.D,) + spatial, 12, 1e-3)
    f = lbm.equilibrium(rho, u, st) * (1.0 + synthetic.random_normal((st.Q,) + spatial, 13, 0.03))
    out = lbm.bgk_collide(f, 0.6, st, F)
    torch.testing.assert_close(lbm.density(out), lbm.density(f), rtol=1e-14, atol=0)
    torch.testing.assert_close(lbm.momentum(out, st), lbm.momentum(f, st) + F, rtol=0, atol=1e-15)


def test_dellar_basis_structure():
    # The non-hydrodynamic weight g is (up to a factor) the fourth-order Hermite
    # polynomial (c_x^2 - 1/3)(c_y^2 - 1/3): w-orthogonal to 1, c, cc, and g on the
    # rest/axis/diagonal velocities is 1, -2, 4 (Dellar 2003).
    st = lbm.stencil("D2Q9")
    M = lbm.dellar_matrix(st)
    assert torch.linalg.matrix_rank(M) == 9
    cls = (st.c ** 2).sum(1)
    g = M[6]
    assert torch.equal(g[cls == 0], torch.tensor([1.0], dtype=torch.float64))
    assert bool((g[cls == 1] == -2).all()) and bool((g[cls == 2] == 4).all())
    # the three non-hydrodynamic rows are w-orthogonal to the six hydrodynamic ones and
    # to each other
    for k in range(6):
        for j in (6, 7, 8):
            assert abs(float((st.w * M[k] * M[j]).sum())) < 1e-15
    for j, l in ((6, 7), (6, 8), (7, 8)):
        assert abs(float((st.w * M[j] * M[l]).sum())) < 1e-15


def test_mrt_equal_times_is_bgk():
    st = lbm.stencil("D2Q9")
    spatial = (6, 7)
    rho, u = synthetic.random_fields(spatial, 2, 91, drho=0.03, umax=0.06)
    f = lbm.equilibrium(rho, u, st) * (1 + synthetic.random_normal((9,) + spatial, 92, 0.02))
    for tau in (0.53, 0.8, 1.4):
        torch.testing.assert_close(lbm.mrt_collide(f, [tau] * 9, st), lbm.bgk_collide(f, tau, st),
                                   rtol=0, atol=2e-15)  # roundoff of the moment-space round trip


def test_mrt_conserves_and_relaxes_each_moment():
    st = lbm.stencil("D2Q9")
    spatial = (5, 4)
    rho, u = synthetic.random_fields(spatial, 2, 93, drho=0.03, umax=0.06)
    f = lbm.equilibrium(rho, u, st) * (1 + synthetic.random_normal((9,) + spatial, 94, 0.02))
    taus = [1.0, 1.0, 1.0, 0.6, 0.6, 0.6, 0.9, 1.3, 1.3]
    out = lbm.mrt_collide(f, taus, st)
    torch.testing.assert_close(lbm.density(out), lbm.density(f), rtol=1e-14, atol=0)
    torch.testing.assert_close(lbm.momentum(out, st), lbm.momentum(f, st), rtol=0, atol=1e-15)
    # the stress relaxes at rate 1/tau_3..5 like BGK with tau = 0.6: the second
    # moment of out equals BGK's
    cf = st.c.to(torch.float64)
    m2 = lambda x: torch.einsum("qa,qb,q...->ab...", cf, cf, x)
    torch.testing.assert_close(m2(out), m2(lbm.bgk_collide(f, 0.6, st)), rtol=0, atol=1e-15)
