"""Pins of the oracle's neural collision (Sec. 3.1): parameter count, reductions to
the plain MRT collision, the equilibrium fixed point, the inputs as moments of the
non-equilibrium part, the affine regime of a ReLU network against a matrix product,
the oddness of a bias-free tanh network, and conservation."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import lbm as olbm
from oracle import neural as onn

ST = olbm.stencil("D2Q9")
SPATIAL = (6, 7)


def _h(seed=3, amp=0.02):
    rho, u = synthetic.random_fields(SPATIAL, 2, seed, drho=0.03, umax=0.06)
    return olbm.equilibrium(rho, u, ST) * (1 + synthetic.random_normal((9,) + SPATIAL, seed + 1, amp))


def _params(seed, w1_scale=1.0, b_scale=1.0, w2_scale=1.0):
    g = np.random.default_rng(seed)
    W1 = g.normal(0, w1_scale, (onn.N_HIDDEN, onn.N_IN))
    b1 = g.normal(0, b_scale, onn.N_HIDDEN)
    W2 = g.normal(0, w2_scale, (onn.N_OUT, onn.N_HIDDEN))
    return torch.from_numpy(np.concatenate([W1.ravel(), b1, W2.ravel()])), (W1, b1, W2)


def test_parameter_count_is_the_papers():
    assert onn.N_PARAMS == 530
    p, (W1, b1, W2) = _params(0)
    a, b, c = onn.split(p)
    assert np.array_equal(a.numpy(), W1) and np.array_equal(b.numpy(), b1) and np.array_equal(c.numpy(), W2)
    with pytest.raises(ValueError):
        onn.split(torch.zeros(529))


@pytest.mark.parametrize("activation", onn.ACTIVATIONS)
def test_zero_network_is_mrt_with_ghost_times_three_halves(activation):
    """All weights zero: t = 0, so tau_6..8 = exp(0) + 1/2 = 3/2 everywhere."""
    h = _h()
    got = onn.collide(h, 0.6, torch.zeros(onn.N_PARAMS), activation, ST)
    ref = olbm.mrt_collide(h, [1, 1, 1, 0.6, 0.6, 0.6, 1.5, 1.5, 1.5], ST)
    assert float((got - ref).abs().max()) < 1e-15


@pytest.mark.parametrize("activation", onn.ACTIVATIONS)
def test_inputs_vanish_at_equilibrium(activation):
    """At h = f^eq the inputs are zero, so the ghost times are exp(W2 act(b1)) + 1/2 for
    any W1 (numpy closed form), and f^eq is a fixed point of the collision."""
    rho, u = synthetic.random_fields(SPATIAL, 2, 9, drho=0.03, umax=0.06)
    feq = olbm.equilibrium(rho, u, ST)
    p, (W1, b1, W2) = _params(1, w1_scale=1e4, w2_scale=0.2)
    x = onn.inputs(feq, ST)
    assert float(x.abs().max()) < 1e-16  # roundoff only: W1 x stays below 1e-12
    act = np.maximum(b1, 0.0) if activation == "relu" else np.tanh(b1)
    want = np.exp(W2 @ act) + 0.5
    got = onn.ghost_taus(feq, p, activation, ST)
    assert np.allclose(got.reshape(3, -1).numpy(), want[:, None], rtol=1e-11, atol=0)
    assert float((onn.collide(feq, 0.6, p, activation, ST) - feq).abs().max()) < 1e-15


def test_inputs_are_moments_of_the_non_equilibrium_part():
    """A perturbation w_i R_k(c_i) along a ghost row R_k of the w-orthogonal basis leaves
    rho and u unchanged, so the inputs are exactly M[3:] applied to it (numpy)."""
    rho, u = synthetic.random_fields(SPATIAL, 2, 5, drho=0.02, umax=0.05)
    feq = olbm.equilibrium(rho, u, ST)
    c = ST.c.numpy().astype(float)
    w = ST.w.numpy()
    gx = (3 * c[:, 0] ** 2 - 1) * (3 * c[:, 1] ** 2 - 1)
    rows = {"N": gx, "Jx": gx * c[:, 0], "Jy": gx * c[:, 1], "xy": c[:, 0] * c[:, 1]}
    M = np.stack([np.ones(9), c[:, 0], c[:, 1], c[:, 0] ** 2, c[:, 0] * c[:, 1], c[:, 1] ** 2, gx, gx * c[:, 0],
                  gx * c[:, 1]])
    for name, R in rows.items():
        eps = 1e-3
        pert = eps * w * R
        assert abs(pert.sum()) < 1e-18 and np.abs(c.T @ pert).max() < 1e-18
        h = feq + torch.from_numpy(pert).reshape(9, 1, 1)
        x = onn.inputs(h, ST).reshape(6, -1).numpy()
        want = M[3:] @ pert
        assert np.allclose(x, want[:, None], atol=1e-15), name


def test_relu_network_in_its_linear_region_is_affine():
    """With biases far above |W1 x| every ReLU unit is active and the network is the
    affine map x -> (W2 W1) x + W2 b1 (numpy matrix products)."""
    h = _h(amp=0.01)
    x = onn.inputs(h, ST).reshape(6, -1).numpy()
    p, (W1, b1, W2) = _params(2, w1_scale=1.0, w2_scale=0.05)
    b1 = np.abs(b1) + 10.0
    p = torch.from_numpy(np.concatenate([W1.ravel(), b1, W2.ravel()]))
    assert np.abs(W1 @ x).max() < 1.0
    t = (W2 @ W1) @ x + (W2 @ b1)[:, None]
    got = onn.ghost_taus(h, p, "relu", ST).reshape(3, -1).numpy()
    assert np.allclose(got, np.exp(t) + 0.5, rtol=1e-13, atol=0)


def test_bias_free_tanh_network_is_odd():
    """b1 = 0 and tanh: t(-x) = -t(x), so (tau(x) - 1/2)(tau(-x) - 1/2) = 1."""
    h = _h()
    rho = olbm.density(h)
    feq = olbm.equilibrium(rho, olbm.momentum(h, ST) / rho, ST)
    mirrored = 2 * feq - h  # same rho and u, non-equilibrium part negated
    p, (W1, b1, W2) = _params(4, w1_scale=3e3, w2_scale=0.2)
    p = torch.from_numpy(np.concatenate([W1.ravel(), np.zeros_like(b1), W2.ravel()]))
    a = onn.ghost_taus(h, p, "tanh", ST) - 0.5
    b = onn.ghost_taus(mirrored, p, "tanh", ST) - 0.5
    # 2 f^eq - h has the same rho and u up to roundoff (~1e-17), which W1 and W2 carry
    # into t at the 1e-12 level
    assert float((a * b - 1).abs().max()) < 1e-10
    assert float((a - 1).abs().max()) > 1e-3  # the network is not trivially zero


@pytest.mark.parametrize("activation", onn.ACTIVATIONS)
def test_collision_conserves_mass_and_momentum(activation):
    h = _h()
    p, _ = _params(6, w1_scale=3e3)
    out = onn.collide(h, 0.55, p, activation, ST)
    assert float((olbm.density(out) - olbm.density(h)).abs().max()) < 1e-15
    assert float((olbm.momentum(out, ST) - olbm.momentum(h, ST)).abs().max()) < 1e-15
    assert float((out - h).abs().max()) > 1e-6
